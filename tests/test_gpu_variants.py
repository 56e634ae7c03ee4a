"""GPU parity of the method's variants against the FP64 oracle (through the C ABI):

- the theta-scheme (Sec. 2, eq:los): Crank-Nicolson and forward Euler trajectories equal the oracle's
  sequential theta-scheme with direct solves;
- MGRIT cycle types (Sec. 3): W- and F-cycles converge to the same trajectory, with the oracle's
  iteration counts;
- the paper's p = 1 solve, one h-multigrid W-cycle (Sec. 4, the paragraph after step 5): spatial solves
  equal dense solves with the oracle's V-cycle counts, and MGRIT trajectories equal the oracle's
  sequential solution;
- Jacobi-preconditioned CG as the spatial solver (the comparison of Sec. 4 and Sec. 5): spatial solves
  equal dense solves with the oracle's iteration counts, MGRIT trajectories equal the oracle's.
"""
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def per_step_max(U, Us):
    """max over time points k >= 1 of ||U_k - Us_k|| / ||Us_k||"""
    num = np.linalg.norm(U[1:] - Us[1:], axis=1)
    den = np.linalg.norm(Us[1:], axis=1)
    return float(np.max(num / np.maximum(den, 1e-300)))


def solver(cfg, theta=1.0, precision=0, tol=1e-10, stol=1e-12, cycle=0, solver_kind=0, coarse=0, maxcyc=100,
           max_iter=100, **so):
    probs = [pm.problem(d["p"], d["n"], d["Nt"], kappa=d["kappa"], T=d["T"], domain=d["domain"], theta=theta)
             for d in cfg["instances"]]
    mo = pm.default_mgrit_opts(cfactor=cfg["m"], max_levels=cfg["max_levels"], coarsest_max=cfg["coarsest_max"],
                               tol=tol, cycle=cycle, max_iter=max_iter)
    sopts = pm.default_solver_opts(precision=precision, spatial_tol=stol, solver=solver_kind, coarse=coarse,
                                   max_vcycles=maxcyc, **so)
    S = pm.Solver(probs, mo, sopts, device=0)
    for i, d in enumerate(cfg["instances"]):
        S.set_source(i, d["src"], d["tkind"])
        if d["init"]:
            S.set_initial_modes(i, d["init"])
    return S


def oracle_seq(d, theta=1.0):
    P = O.Problem(d["p"], d["n"], d["domain"])
    F = P.load_vector(d["src"])
    u0 = P.project(d["init"]) if d["init"] else np.zeros(P.ndof)
    return P, F, u0, P.sequential(d["kappa"], d["T"], d["Nt"], F, d["tkind"], u0, theta=theta)


# ---------------------------------------------------------------------------------------------
# spatial solves
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("p,n,domain,precision", [
    (2, 16, 0, 0), (3, 32, 1, 0), (3, 12, 0, 1), (4, 9, 0, 0), (2, 64, 1, 1), (5, 24, 0, 0)])
def test_phi_hmg_matches_dense_and_oracle_counts(torch, p, n, domain, precision):
    """p = 1 solve by one h-multigrid W-cycle: every solve reaches the spatial tolerance, equals the dense
    solve, and takes the oracle's number of V-cycles (same algorithm, rounding aside)."""
    say(f"case phi h-multigrid p={p} n={n} domain={domain} precision={precision}")
    cfg = W.small("x", p, n, 16, domain=domain)
    S = solver(cfg, precision=precision, coarse=1)
    P = O.Problem(p, n, domain)
    say(f"  h-levels {P.hmg_levels()}")
    rng = np.random.default_rng(7 * p + n)
    nrhs = 5
    for level in range(S.dims()[2]):
        dt = 0.1 / 16 * 4 ** level
        A = P.dense("M") + dt * P.dense("K")
        B = rng.standard_normal((nrhs, P.ndof))
        b = torch.tensor(B, device="cuda")
        x = torch.zeros_like(b)
        vc = torch.zeros(nrhs, dtype=torch.int32, device="cuda")
        S.phi(0, level, b, x, vc)
        X = x.cpu().numpy()
        for j in range(nrhs):
            r = np.linalg.norm(B[j] - A @ X[j]) / np.linalg.norm(B[j])
            assert r <= 1.0000001e-12, (level, j, r)
            assert rel(X[j], np.linalg.solve(A, B[j])) < 1e-9
            rc, _, cyc = P.pmg_solve(1.0, dt, B[j], tol=1e-12, prec=precision, coarse=1)
            assert rc == 0
            assert abs(int(vc[j]) - cyc) <= 1, (level, j, int(vc[j]), cyc)


@pytest.mark.parametrize("p,n,domain", [(2, 16, 0), (3, 12, 1), (4, 10, 0), (5, 8, 1)])
def test_phi_cg_matches_dense_and_oracle_counts(torch, p, n, domain):
    """Jacobi-preconditioned CG: every solve reaches the tolerance, equals the dense solve, and takes the
    oracle's number of iterations to within rounding (a few per cent)."""
    say(f"case phi CG p={p} n={n} domain={domain}")
    cfg = W.small("x", p, n, 16, domain=domain)
    S = solver(cfg, solver_kind=1, maxcyc=5000)
    P = O.Problem(p, n, domain)
    rng = np.random.default_rng(11 * p + n)
    nrhs = 4
    for level in range(S.dims()[2]):
        dt = 0.1 / 16 * 4 ** level
        A = P.dense("M") + dt * P.dense("K")
        B = rng.standard_normal((nrhs, P.ndof))
        X0 = np.zeros_like(B)
        X0[2] = rng.standard_normal(P.ndof)
        b = torch.tensor(B, device="cuda")
        x = torch.tensor(X0, device="cuda")
        vc = torch.zeros(nrhs, dtype=torch.int32, device="cuda")
        S.phi(0, level, b, x, vc)
        X = x.cpu().numpy()
        for j in range(nrhs):
            r = np.linalg.norm(B[j] - A @ X[j]) / np.linalg.norm(B[j])
            assert r <= 1.0000001e-12, (level, j, r)
            assert rel(X[j], np.linalg.solve(A, B[j])) < 1e-8
            rc, _, it = P.pmg_solve(1.0, dt, B[j], x0=X0[j], tol=1e-12, solver=1, maxcyc=5000)
            assert rc == 0
            assert abs(int(vc[j]) - it) <= max(2, 0.05 * it), (level, j, int(vc[j]), it)


# ---------------------------------------------------------------------------------------------
# time stepping variants
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("domain", [0, 1])
def test_mgrit_crank_nicolson(torch, domain):
    cfg = W.small("x", 3, 12, 64, domain=domain)
    say(f"case MGRIT Crank-Nicolson p=3 n=12 N_t=64 domain={domain}")
    S = solver(cfg, theta=0.5, tol=1e-12, stol=1e-13)
    (U,), st = S.solve_mgrit()
    d = cfg["instances"][0]
    P, F, u0, Us = oracle_seq(d, theta=0.5)
    U = U.cpu().numpy()
    e, ek = rel(U, Us), per_step_max(U, Us)
    say(f"  eps={e:.2e} per-step max={ek:.2e} iters={st['mgrit_iters']}")
    assert e <= EPS and ek <= EPS
    r = P.mgrit(d["kappa"], d["T"], d["Nt"], F, d["tkind"], u0, m=cfg["m"], coarsest_max=cfg["coarsest_max"],
                tol=1e-12, stol=1e-13, theta=0.5)
    assert abs(st["mgrit_iters"] - r["iters"]) <= 1


def test_manufactured_crank_nicolson_sequential(torch):
    """C1's manufactured problem with Crank-Nicolson (theta-weighted source), sequential stepping"""
    cfg = W.config("heat-p2-h16-Nt128")
    say("case sequential Crank-Nicolson heat-p2-h16-Nt128")
    S = solver(cfg, theta=0.5, stol=1e-13)
    (U,), _ = S.solve_sequential()
    _, _, _, Us = oracle_seq(cfg["instances"][0], theta=0.5)
    U = U.cpu().numpy()
    e, ek = rel(U, Us), per_step_max(U, Us)
    say(f"  eps={e:.2e} per-step max={ek:.2e}")
    assert e <= EPS and ek <= EPS


def test_mgrit_forward_euler(torch):
    """explicit steps on every level: kappa dt_l lambda_max of the pencil (K, M) stays below 2 on the
    coarsest level (p = 2, n = 3, T = 0.05, N_t = 1024, m = 2, three levels)"""
    d = dict(p=2, n=3, domain=0, kappa=1.0, T=0.05, Nt=1024, src=[(1, 1, 1.0), (2, 1, -0.5)], tkind=0,
             init=[(1, 2, 0.7)])
    P = O.Problem(2, 3, 0)
    import scipy.linalg as sl
    lmax = sl.eigh(P.dense("K"), P.dense("M"), eigvals_only=True).max()
    assert 1.0 * (0.05 / 1024) * 4 * lmax < 2.0
    cfg = dict(instances=[d], m=2, max_levels=3, coarsest_max=1)
    say("case MGRIT forward Euler p=2 n=3 N_t=1024 m=2 three levels")
    S = solver(cfg, theta=0.0, tol=1e-12, stol=1e-13)
    (U,), st = S.solve_mgrit()
    _, _, _, Us = oracle_seq(d, theta=0.0)
    U = U.cpu().numpy()
    e, ek = rel(U, Us), per_step_max(U, Us)
    say(f"  eps={e:.2e} per-step max={ek:.2e} iters={st['mgrit_iters']}")
    assert e <= EPS and ek <= EPS


@pytest.mark.parametrize("cycle", [1, 2])
def test_mgrit_cycle_types(torch, cycle):
    """W- (1) and F-cycles (2) on four levels: the oracle's sequential trajectory, the oracle's MGRIT
    iteration count (same cycle), and no more iterations than the V-cycle"""
    cfg = W.small("x", 2, 8, 256, domain=0)
    cfg["coarsest_max"] = 4
    d = cfg["instances"][0]
    say(f"case MGRIT cycle {cycle} p=2 n=8 N_t=256 m=4")
    S = solver(cfg, cycle=cycle, tol=1e-12, stol=1e-13)
    (U,), st = S.solve_mgrit()
    assert S.dims()[2] == 4
    P, F, u0, Us = oracle_seq(d)
    U = U.cpu().numpy()
    e, ek = rel(U, Us), per_step_max(U, Us)
    r = P.mgrit(d["kappa"], d["T"], d["Nt"], F, d["tkind"], u0, m=4, coarsest_max=4, tol=1e-12, stol=1e-13,
                cycle=cycle)
    rv = P.mgrit(d["kappa"], d["T"], d["Nt"], F, d["tkind"], u0, m=4, coarsest_max=4, tol=1e-12, stol=1e-13,
                 cycle=0)
    say(f"  eps={e:.2e} per-step max={ek:.2e} iters={st['mgrit_iters']} oracle {r['iters']} (V: {rv['iters']})")
    assert e <= EPS and ek <= EPS
    assert abs(st["mgrit_iters"] - r["iters"]) <= 1
    assert st["mgrit_iters"] <= rv["iters"] + 1


def test_mgrit_cycle_types_two_level_coincide(torch):
    cfg = W.small("x", 3, 10, 64, domain=1)
    cfg["max_levels"] = 2
    res = []
    for c in (0, 1, 2):
        S = solver(cfg, cycle=c)
        (U,), st = S.solve_mgrit()
        res.append((U.cpu().numpy(), st["mgrit_iters"]))
        S.close()
    for U, it in res[1:]:
        assert it == res[0][1] and np.array_equal(U, res[0][0])


# ---------------------------------------------------------------------------------------------
# MGRIT with the paper's p = 1 h-multigrid and with CG
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("name,precision", [("heat-p2-h16-Nt128", 0), ("heat-p3-h64-Nt1024", 0),
                                            ("heat-p5-h64-Nt1024", 1)])
def test_mgrit_hmg_coarse_solve(torch, name, precision):
    cfg = W.config(name)
    say(f"case MGRIT {name} with the h-multigrid p = 1 solve, precision {precision}")
    st = {}
    U = {}
    for coarse in (0, 1):
        S = solver(cfg, precision=precision, coarse=coarse)
        (u,), st[coarse] = S.solve_mgrit()
        U[coarse] = u.cpu().numpy()
        S.close()
    _, _, _, Us = oracle_seq(cfg["instances"][0])
    e, ek = rel(U[1], Us), per_step_max(U[1], Us)
    say(f"  eps={e:.2e} per-step max={ek:.2e}; V-cycles per solve exact {st[0]['vcycles'] / st[0]['phi_calls']:.3f}"
        f" h-MG {st[1]['vcycles'] / st[1]['phi_calls']:.3f}; iters {st[0]['mgrit_iters']} / {st[1]['mgrit_iters']}"
        f"; t {st[0]['t_solve_s']:.2f} / {st[1]['t_solve_s']:.2f} s")
    assert e <= EPS and ek <= EPS
    assert abs(st[1]["mgrit_iters"] - st[0]["mgrit_iters"]) <= 1


def test_mgrit_hmg_annulus(torch):
    cfg = W.small("x", 4, 32, 128, domain=1)
    say("case MGRIT annulus p=4 n=32 N_t=128 with the h-multigrid p = 1 solve")
    S = solver(cfg, coarse=1, tol=1e-12, stol=1e-13)
    (U,), st = S.solve_mgrit()
    _, _, _, Us = oracle_seq(cfg["instances"][0])
    U = U.cpu().numpy()
    e, ek = rel(U, Us), per_step_max(U, Us)
    say(f"  eps={e:.2e} per-step max={ek:.2e} iters={st['mgrit_iters']} V/solve {st['vcycles'] / st['phi_calls']:.3f}")
    assert e <= EPS and ek <= EPS


@pytest.mark.parametrize("domain", [0, 1])
def test_mgrit_cg_spatial_solver(torch, domain):
    cfg = W.small("x", 3, 16, 64, domain=domain)
    say(f"case MGRIT with CG spatial solves p=3 n=16 N_t=64 domain={domain}")
    S = solver(cfg, solver_kind=1, maxcyc=5000, tol=1e-12, stol=1e-13)
    (U,), st = S.solve_mgrit()
    d = cfg["instances"][0]
    P, F, u0, Us = oracle_seq(d)
    U = U.cpu().numpy()
    e, ek = rel(U, Us), per_step_max(U, Us)
    r = P.mgrit(d["kappa"], d["T"], d["Nt"], F, d["tkind"], u0, m=cfg["m"], coarsest_max=cfg["coarsest_max"],
                tol=1e-12, stol=1e-13, solver=1, maxcyc=5000)
    say(f"  eps={e:.2e} per-step max={ek:.2e} iters={st['mgrit_iters']} (oracle {r['iters']}) "
        f"CG it/solve {st['vcycles'] / st['phi_calls']:.1f} (oracle {r['cycles'] / r['solves']:.1f})")
    assert e <= EPS and ek <= EPS
    assert abs(st["mgrit_iters"] - r["iters"]) <= 1


def test_cg_versus_pmg_by_degree(torch):
    """The paper's comparison (Sec. 5): at h = 2^-6 CG iterations per solve grow quickly with p while
    p-multigrid V-cycles per solve stay flat.  Both solvers reach the oracle's trajectory (MGRIT to
    1e-12, spatial solves to 1e-13: CG's recursively updated residual drifts from the true one as the
    conditioning worsens with p)."""
    rows = []
    for p in (2, 3, 4, 5):
        d = dict(p=p, n=64, domain=0, kappa=1.0, T=0.1 * 128 / 1024, Nt=128, src=W.random_modes(2107), tkind=0,
                 init=[])
        cfg = dict(instances=[d], m=8, max_levels=12, coarsest_max=8)
        _, _, _, Us = oracle_seq(d)
        row = [p]
        for kind in (0, 1):
            S = solver(cfg, solver_kind=kind, maxcyc=5000, tol=1e-12, stol=1e-13)
            (U,), st = S.solve_mgrit()
            U = U.cpu().numpy()
            e, ek = rel(U, Us), per_step_max(U, Us)
            assert e <= EPS and ek <= EPS, (p, kind, e, ek)
            row += [st["vcycles"] / st["phi_calls"], st["t_solve_s"]]
            S.close()
        rows.append(row)
        say(f"  p={p}: p-MG {row[1]:.2f} V-cycles/solve {row[2]:.3f} s; CG {row[3]:.1f} it/solve {row[4]:.3f} s")
    pmg = [r[1] for r in rows]
    cg = [r[3] for r in rows]
    assert max(pmg) <= 2.5
    assert cg[3] > 2 * cg[0] and all(cg[i + 1] > cg[i] for i in range(3))
