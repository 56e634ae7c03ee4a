"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

The bar: every trajectory matches the oracle's sequential implicit Euler with direct solves (the
plain definition of what MGRIT converges to, eq:mgrit) to 1e-10 relative in the discrete L2 norm
over all time points, and every spatial solve matches a dense direct solve."""
import sys

import numpy as np
import pytest

try:  # imported at collection time so a slow first import is not charged to a test's timeout
    import torch as _torch  # noqa: F401
except Exception:  # pragma: no cover
    _torch = None

import oracle as O
import paper_2107_05337_amd as pm
from paper_2107_05337_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a visible MI355X"
    return T


def make_solver(cfg, precision=0, guess=2, trsv_block=0, tol=1e-10, stol=1e-12, autotune=0, ctol=0.0, lds_mask=0,
                **mo):
    probs = [pm.problem(d["p"], d["n"], d["Nt"], kappa=d["kappa"], T=d["T"], domain=d["domain"])
             for d in cfg["instances"]]
    mopts = pm.default_mgrit_opts(cfactor=cfg["m"], max_levels=cfg["max_levels"], coarsest_max=cfg["coarsest_max"],
                                  tol=tol, **mo)
    sopts = pm.default_solver_opts(precision=precision, guess=guess, trsv_block=trsv_block, spatial_tol=stol,
                                   autotune=autotune, coarse_tol=ctol, lds_mask=lds_mask)
    S = pm.Solver(probs, mopts, sopts, device=0)
    for i, d in enumerate(cfg["instances"]):
        S.set_source(i, d["src"], d["tkind"])
        if d["init"]:
            S.set_initial_modes(i, d["init"])
    return S


def oracle_sequential(d, nsteps=None):
    P = O.Problem(d["p"], d["n"], d["domain"])
    F = P.load_vector(d["src"])
    u0 = P.project(d["init"]) if d["init"] else np.zeros(P.ndof)
    Nt = d["Nt"] if nsteps is None else nsteps
    T = d["T"] * Nt / d["Nt"]
    return P.sequential(d["kappa"], T, Nt, F, d["tkind"], u0)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("p,n,domain,precision,blk", [
    (2, 8, 0, 0, -1), (3, 12, 0, 0, 1), (3, 12, 1, 0, -1), (4, 10, 0, 1, -1), (2, 16, 1, 1, 1), (5, 9, 0, 0, 7),
    (3, 12, 1, 0, 0), (4, 10, 0, 1, 0), (5, 70, 0, 0, 0), (3, 62, 0, 1, 0)])
def test_phi_matches_dense_solve(torch, p, n, domain, precision, blk):
    say(f"case phi p={p} n={n} domain={domain} precision={precision} block={blk}")
    cfg = W.small("x", p, n, 16, domain=domain)
    S = make_solver(cfg, precision=precision, trsv_block=blk)
    P = O.Problem(p, n, domain)
    rng = np.random.default_rng(p * 100 + n)
    nrhs = 7
    for level in range(S.dims()[2]):
        dt = 0.1 / 16 * 4 ** level
        A = P.dense("M") + dt * P.dense("K")
        B = rng.standard_normal((nrhs, P.ndof))
        B[3] = 0.0  # a zero right-hand side is solved by the zero guess in zero cycles
        X0 = np.zeros_like(B)
        X0[1] = rng.standard_normal(P.ndof)  # a non-zero initial guess
        b = torch.tensor(B, device="cuda")
        x = torch.tensor(X0, device="cuda")
        vc = torch.zeros(nrhs, dtype=torch.int32, device="cuda")
        S.phi(0, level, b, x, vc)
        X = x.cpu().numpy()
        for j in range(nrhs):
            if j == 3:
                assert np.all(X[j] == 0.0) and int(vc[j]) == 0
                continue
            r = np.linalg.norm(B[j] - A @ X[j]) / np.linalg.norm(B[j])
            assert r <= 1.0000001e-12, (level, j, r)
            xe = np.linalg.solve(A, B[j])
            assert rel(X[j], xe) < 1e-9
            assert 1 <= int(vc[j]) <= 20


def test_mgrit_two_level_manufactured(torch):
    cfg = W.config("heat-p2-h16-Nt128")
    say("case mgrit heat-p2-h16-Nt128 (two-level, m=4)")
    S = make_solver(cfg)
    (U,), st = S.solve_mgrit()
    Us = oracle_sequential(cfg["instances"][0])
    eps = rel(U.cpu().numpy(), Us)
    say(f"  eps={eps:.3e} iters={st['mgrit_iters']} vcycles={st['vcycles']}")
    assert eps <= EPS
    # same algorithm as the oracle's MGRIT: same iteration count
    d = cfg["instances"][0]
    P = O.Problem(d["p"], d["n"], 0)
    r = P.mgrit(d["kappa"], d["T"], d["Nt"], P.load_vector(d["src"]), d["tkind"], P.project(d["init"]), m=4,
                max_levels=2, tol=1e-10)
    assert abs(st["mgrit_iters"] - r["iters"]) <= 1
    assert st["res_hist"][0] == 1.0 and st["res_hist"][-1] <= 1e-10


@pytest.mark.parametrize("p", [3, 4, 5])
def test_mgrit_multilevel_full_size(torch, p):
    name = f"heat-p{p}-h64-Nt1024"
    say(f"case mgrit {name}")
    cfg = W.config(name)
    S = make_solver(cfg)
    assert S.dims()[2] == 4  # 1024 -> 128 -> 16 -> 2
    (U,), st = S.solve_mgrit()
    Us = oracle_sequential(cfg["instances"][0])
    eps = rel(U.cpu().numpy(), Us)
    say(f"  eps={eps:.3e} iters={st['mgrit_iters']} vcycles={st['vcycles']} t={st['t_solve_s']:.3f}s")
    assert eps <= EPS
    assert 5 <= st["mgrit_iters"] <= 15


def test_mgrit_fp32_refined_full_size(torch):
    name = "heat-p3-h64-Nt1024"
    say(f"case mgrit {name} FP32 V-cycle in FP64 refinement")
    cfg = W.config(name)
    S = make_solver(cfg, precision=1)
    (U,), st = S.solve_mgrit()
    Us = oracle_sequential(cfg["instances"][0])
    eps = rel(U.cpu().numpy(), Us)
    say(f"  eps={eps:.3e} iters={st['mgrit_iters']} vcycles={st['vcycles']} t={st['t_solve_s']:.3f}s")
    assert eps <= EPS


@pytest.mark.parametrize("precision", [0, 1])
def test_sequential_matches_oracle(torch, precision):
    cfg = W.small("x", 3, 16, 40, domain=1)
    say(f"case sequential annulus p=3 n=16 Nt=40 precision={precision}")
    S = make_solver(cfg, precision=precision)
    (U,), st = S.solve_sequential()
    Us = oracle_sequential(cfg["instances"][0])
    assert rel(U.cpu().numpy(), Us) <= EPS
    assert st["phi_calls"] == 40


@pytest.mark.parametrize("Nt,m", [(37, 4), (1, 4), (9, 8), (64, 2)])
def test_mgrit_ragged_and_degenerate(torch, Nt, m):
    say(f"case mgrit ragged Nt={Nt} m={m}")
    cfg = W.small("x", 2, 8, Nt)
    cfg["m"] = m
    S = make_solver(cfg, tol=1e-12)
    (U,), st = S.solve_mgrit()
    Us = oracle_sequential(cfg["instances"][0])
    assert rel(U.cpu().numpy(), Us) <= EPS


def test_heterogeneous_batch(torch):
    say("case mgrit heterogeneous batch of 4 instances")
    insts = [
        dict(p=2, n=8, domain=0, kappa=0.3, T=0.1, Nt=64, src=W.random_modes(11, 3, 4), tkind=0, init=[]),
        dict(p=3, n=16, domain=1, kappa=2.0, T=0.1, Nt=64, src=W.random_modes(12, 3, 4), tkind=0, init=[]),
        dict(p=4, n=8, domain=0, kappa=1.0, T=0.1, Nt=64, src=W.random_modes(13, 3, 4), tkind=1,
             init=[(1, 1, 1.0)]),
        dict(p=5, n=12, domain=1, kappa=5.0, T=0.1, Nt=64, src=W.random_modes(14, 3, 4), tkind=0, init=[]),
    ]
    cfg = dict(instances=insts, m=4, max_levels=12, coarsest_max=4)
    S = make_solver(cfg, tol=1e-11)
    U, st = S.solve_mgrit()
    for i, d in enumerate(insts):
        eps = rel(U[i].cpu().numpy(), oracle_sequential(d))
        say(f"  instance {i}: eps={eps:.3e}")
        assert eps <= EPS


def test_deterministic(torch):
    say("case determinism heat-p2-h16-Nt128")
    cfg = W.config("heat-p2-h16-Nt128")
    S = make_solver(cfg)
    (U1,), _ = S.solve_mgrit()
    (U2,), _ = S.solve_mgrit()
    assert torch.equal(U1, U2)


@pytest.mark.parametrize("hetero", [False, True])
def test_graph_replay_matches_eager(torch, hetero):
    """The captured MGRIT iteration (kernels only) replayed every iteration gives bitwise the eager
    result, also on a second solve that replays the cached graph after unrelated eager work."""
    if hetero:  # two launch groups: the capture contains the fork / join across group streams
        insts = [dict(p=2, n=8, domain=0, kappa=1.0, T=0.1, Nt=128, src=W.random_modes(21, 3, 4), tkind=0, init=[]),
                 dict(p=4, n=128, domain=1, kappa=0.5, T=0.1, Nt=128, src=W.random_modes(22, 3, 4), tkind=0,
                      init=[])]
        cfg = dict(instances=insts, m=4, max_levels=4, coarsest_max=4)
    else:
        cfg = W.small("x", 3, 16, 256)
        cfg["m"], cfg["max_levels"], cfg["coarsest_max"] = 4, 4, 4
    say(f"case graph replay hetero={hetero}")
    Se = make_solver(cfg, tol=1e-12)
    Ue, ste = Se.solve_mgrit()
    Sg = make_solver(cfg, tol=1e-12, use_graph=1)
    if hetero:
        assert Sg.group_info(0)["groups"] == 2
    outs = Sg.alloc_trajectories()
    Ug, stg = Sg.solve_mgrit(outs)
    first = [u.clone() for u in Ug]
    junk = torch.randn(1 << 20, device="cuda")
    junk = (junk * 2).sum()  # eager work between the solves
    torch.cuda.synchronize()
    Ug2, stg2 = Sg.solve_mgrit(outs)
    say(f"  iters eager {ste['mgrit_iters']} graph {stg['mgrit_iters']} / {stg2['mgrit_iters']}")
    assert ste["mgrit_iters"] == stg["mgrit_iters"] == stg2["mgrit_iters"] >= 2
    assert ste["phi_calls"] == stg["phi_calls"] and ste["vcycles"] == stg["vcycles"]
    for a, b, c in zip(Ue, first, Ug2):
        assert torch.equal(a, b) and torch.equal(a, c)
    for i, d in enumerate(cfg["instances"]):
        assert rel(first[i].cpu().numpy(), oracle_sequential(d)) <= EPS


def test_learned_mgrit_two_launch_groups(torch):
    """MGRIT with the learned guess over two launch groups, one of which holds no instance the network
    predicts (more than 64 elements per direction): that group relaxes whole on its own stream while
    the other goes step position by position. Both reach the oracle's trajectory, and the instance
    the network does not predict is bitwise the one of a solve without the network."""
    insts = [dict(p=2, n=8, domain=0, kappa=1.0, T=0.1, Nt=128, src=W.random_modes(21, 3, 4), tkind=0, init=[]),
             dict(p=4, n=128, domain=1, kappa=0.5, T=0.1, Nt=128, src=W.random_modes(22, 3, 4), tkind=0, init=[])]
    cfg = dict(instances=insts, m=4, max_levels=4, coarsest_max=4)
    say("case learned MGRIT over two launch groups")
    S = make_solver(cfg, guess=3, tol=1e-12)
    assert S.group_info(0)["groups"] == 2
    S.net_load(W.net_init(3))
    U, st = S.solve_mgrit()
    S2 = make_solver(cfg, guess=2, tol=1e-12)
    U2, st2 = S2.solve_mgrit()
    say(f"  iters learned {st['mgrit_iters']} previous-iterate {st2['mgrit_iters']}; "
        f"V-cycles {st['vcycles']} / {st2['vcycles']}")
    assert torch.equal(U[1], U2[1])
    for i, d in enumerate(insts):
        assert rel(U[i].cpu().numpy(), oracle_sequential(d)) <= EPS


@pytest.mark.parametrize("graph", [0, 1])
def test_batched_instances_stop_on_their_own(torch, graph):
    """Each instance of a batch stops at its own MGRIT tolerance (Sec. 3's stopping criterion is
    per problem): the faster instance keeps its iterate while the slower one iterates on, so the
    batch returns what each instance's solve alone returns, with the same number of solves."""
    fast = W.small("x", 3, 12, 64, kappa=0.05)["instances"][0]
    slow = W.small("x", 3, 12, 64, kappa=1.0)["instances"][0]

    def run(insts, tol=1e-6):
        cfg = dict(instances=insts, m=4, max_levels=12, coarsest_max=4)
        U, st = make_solver(cfg, tol=tol, use_graph=graph).solve_mgrit()
        return [u.cpu().numpy() for u in U], st

    say(f"case per-instance stop graph={graph}")
    Ub, stb = run([fast, slow])
    (Uf,), stf = run([fast])
    (Us,), sts = run([slow])
    (Uf9,), _ = run([fast], tol=1e-9)
    gap = rel(Uf, Uf9)
    say(f"  iters fast {stf['mgrit_iters']} slow {sts['mgrit_iters']} batch {stb['mgrit_iters']}; "
        f"diff fast {rel(Ub[0], Uf):.1e} slow {rel(Ub[1], Us):.1e}; one more tolerance decade moves fast by {gap:.1e}")
    assert stf["mgrit_iters"] < sts["mgrit_iters"] == stb["mgrit_iters"]
    assert gap > 1e-9  # iterating the fast instance on would be seen below
    assert rel(Ub[0], Uf) <= 1e-13 and rel(Ub[1], Us) <= 1e-13
    assert stb["phi_calls"] == stf["phi_calls"] + sts["phi_calls"]
    assert stb["vcycles"] == stf["vcycles"] + sts["vcycles"]


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_same_result(torch, precision):
    """The autotuner only moves work vectors between LDS and global scratch: same results."""
    name = "heat-p3-h64-Nt1024"
    cfg = W.config(name)
    cfg["instances"][0]["Nt"] = 128
    cfg["instances"][0]["T"] = 0.1 / 8
    say(f"case autotune precision={precision}")
    S0 = make_solver(cfg, precision=precision)
    (U0,), st0 = S0.solve_mgrit()
    S1 = make_solver(cfg, precision=precision, autotune=1)
    gi = S1.group_info(0)
    say(f"  default {S0.group_info(0)['lds_mask']} tuned {gi['lds_mask']} ({gi['lds_bytes']} B)")
    (U1,), st1 = S1.solve_mgrit()
    assert gi["lds_mask"] & 1
    if (gi["lds_mask"] | gi["lds_mask_wide"]) & (32 | 64):
        # the 8-lanes-per-row builds sum each triangular-solve row in another order (and the
        # 1024-thread one the workgroup over 16 waves): the same solves up to rounding
        assert rel(U1.cpu().numpy(), U0.cpu().numpy()) <= 1e-11
        assert abs(st1["vcycles"] - st0["vcycles"]) <= 0.02 * st0["vcycles"]
    else:
        assert torch.equal(U0, U1) and st0["vcycles"] == st1["vcycles"]


@pytest.mark.parametrize("mask,p,n,precision", [(3 | 16, 5, 64, 1), (1 | 16, 5, 64, 1), (3, 5, 64, 1), (2, 5, 64, 1),
                                                 (2, 3, 80, 1), (2, 5, 64, 0), (2, 3, 80, 0)])
def test_forced_placement_same_result(torch, mask, p, n, precision):
    """Forced LDS placements compute the same arithmetic: bitwise the same trajectory and V-cycle
    count as the default placement.  Covers the FP32 kernel build for two workgroups per CU (mask
    bit 16) and y in global memory (mask 2), where the triangular solves read the grid lines they
    couple to from an LDS window.  At n = 80 the 81-row grid lines are split into two blocks, so
    blocks straddle lines."""
    cfg = W.config(f"heat-p{p}-h64-Nt1024")
    d = cfg["instances"][0]
    d["n"], d["Nt"], d["T"] = n, 64, 1.0 / 16
    say(f"case forced placement {mask} p={p} n={n} N_t=64 precision {precision}")
    S0 = make_solver(cfg, precision=precision)
    (U0,), st0 = S0.solve_mgrit()
    S1 = make_solver(cfg, precision=precision, lds_mask=mask)
    gi = S1.group_info(0)
    say(f"  default {S0.group_info(0)['lds_mask']} forced {gi['lds_mask']} ({gi['lds_bytes']} B)")
    assert gi["lds_mask"] == mask
    (U1,), st1 = S1.solve_mgrit()
    assert torch.equal(U0, U1) and st0["vcycles"] == st1["vcycles"]


@pytest.mark.parametrize("precision,mask", [(1, 15 | 32), (0, 15 | 32), (1, 1 | 32), (1, 15 | 64), (0, 15 | 64),
                                            (1, 1 | 64), (0, 3 | 64)])
def test_1024_thread_build(torch, precision, mask):
    """The kernel builds with 8 lanes per triangular-solve row (slot tables in that layout): 1024
    threads (mask bit 32) and 512 threads with 64 row slots (bit 64) reach the oracle's sequential
    implicit Euler to the same 1e-10 as the default build."""
    name = "heat-p5-h64-Nt1024"
    cfg = W.config(name)
    d = cfg["instances"][0]
    d["Nt"], d["T"] = 64, 1.0 / 16
    say(f"case 1024-thread build mask {mask} precision {precision} p=5 n=64 N_t=64")
    S = make_solver(cfg, precision=precision, lds_mask=mask)
    gi = S.group_info(0)
    assert gi["lds_mask"] == mask and gi["lds_mask_wide"] == mask
    (U,), st = S.solve_mgrit()
    P = O.Problem(d["p"], d["n"], d["domain"])
    Us = P.sequential(d["kappa"], d["T"], d["Nt"], P.load_vector(d["src"]), d["tkind"], np.zeros(P.ndof))
    e = rel(U.cpu().numpy(), Us)
    say(f"  iters {st['mgrit_iters']} V-cycles {st['vcycles']} eps {e:.2e}")
    assert e <= 1e-10


@pytest.mark.parametrize("precision", [0, 1])
def test_coarse_tolerance(torch, precision):
    """Looser spatial solves on the coarse levels: same converged answer, same iteration count as
    the oracle's MGRIT with the same coarse tolerance."""
    cfg = W.small("x", 3, 16, 512)
    cfg["m"], cfg["max_levels"], cfg["coarsest_max"] = 8, 12, 8
    d = cfg["instances"][0]
    say(f"case coarse tolerance 1e-6 precision={precision}")
    S = make_solver(cfg, precision=precision, tol=1e-11, ctol=1e-6)
    (U,), st = S.solve_mgrit()
    assert rel(U.cpu().numpy(), oracle_sequential(d)) <= EPS
    P = O.Problem(d["p"], d["n"], 0)
    r = P.mgrit(d["kappa"], d["T"], d["Nt"], P.load_vector(d["src"]), d["tkind"], P.project(d["init"]), m=8,
                tol=1e-11, ctol=1e-6)
    S0 = make_solver(cfg, precision=precision, tol=1e-11)
    _, st0 = S0.solve_mgrit()
    say(f"  iters {st['mgrit_iters']} (oracle {r['iters']}), V-cycles {st['vcycles']} vs {st0['vcycles']} at 1e-12")
    assert abs(st["mgrit_iters"] - r["iters"]) <= 1
    assert st["vcycles"] < st0["vcycles"]


def test_w8_build_needs_64_row_levels(torch):
    """The 512-thread 8-lane build has 64 row slots: with one grid line of 67 rows per block (p = 5,
    n = 64) the forced placement is refused at create, and the autotuner leaves that build out."""
    cfg = W.config("heat-p5-h64-Nt1024")
    cfg["instances"][0]["Nt"] = 16
    say("case 8-lane 512-thread build with 67-row levels")
    with pytest.raises(pm.PmgritError) as e:
        make_solver(cfg, trsv_block=-1, lds_mask=15 | 64)
    assert e.value.code == -1
    S = make_solver(cfg, trsv_block=-1, autotune=1)
    gi = S.group_info(0)
    assert not ((gi["lds_mask"] | gi["lds_mask_wide"]) & 64)
    S.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_window_mode_slab_tables(torch, precision):
    """An instance too large for LDS (p = 3, n = 150: window mode by default, 128-row blocks) in FP64 and
    FP32-refined: the triangular solves run over slab tables (each level's dense rows copied to LDS in
    8 KB chunks, 16-bit window columns) and the trajectory reaches the oracle's."""
    cfg = W.small("x", 3, 150, 16)
    d = cfg["instances"][0]
    say(f"case window mode, slab tables, p=3 n=150 N_t=16 precision {precision}")
    P = O.Problem(d["p"], d["n"], d["domain"])
    Us = P.sequential(d["kappa"], d["T"], d["Nt"], P.load_vector(d["src"]), d["tkind"], P.project(d["init"]))
    S = make_solver(cfg, precision=precision, tol=1e-12, stol=1e-13)
    sch = S.host_schedule()
    gi = S.group_info(0)
    (U,), st = S.solve_mgrit()
    e = rel(U.cpu().numpy(), Us)
    say(f"  block {sch['block_size']} levels {sch['levels']} mask {gi['lds_mask']}: iters {st['mgrit_iters']} "
        f"V-cycles {st['vcycles']} eps {e:.2e}")
    assert gi["lds_mask"] & 1 == 0 and sch["block_size"] == 128
    assert e <= 1e-10
    S.close()


def test_window_mode_128_row_blocks(torch):
    """FP32 triangular solves in window mode (y in global memory, mask 2) with 128-row blocks (the block
    size instances too large for LDS get): the trajectory reaches the oracle's, as with the default
    placement and 64-row blocks."""
    cfg = W.small("x", 3, 130, 16)
    d = cfg["instances"][0]
    say("case window mode, 128-row blocks, p=3 n=130 N_t=16 FP32")
    P = O.Problem(d["p"], d["n"], d["domain"])
    Us = P.sequential(d["kappa"], d["T"], d["Nt"], P.load_vector(d["src"]), d["tkind"], P.project(d["init"]))
    for blk, mask in ((128, 2), (0, 0)):
        S = make_solver(cfg, precision=1, trsv_block=blk, lds_mask=mask, tol=1e-12, stol=1e-13)
        sch = S.host_schedule()
        (U,), st = S.solve_mgrit()
        e = rel(U.cpu().numpy(), Us)
        say(f"  block {sch['block_size']} levels {sch['levels']} mask {S.group_info(0)['lds_mask']}: "
            f"iters {st['mgrit_iters']} V-cycles {st['vcycles']} eps {e:.2e}")
        assert e <= 1e-10
        S.close()
