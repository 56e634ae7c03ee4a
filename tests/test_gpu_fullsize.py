"""GPU parity at full size: the mixed-precision configuration (p = 4, h = 2^-7, N_t = 2048) and the
heterogeneous batch of 16 instances (h 2^-5 .. 2^-8, p 2 .. 5, square and quarter annulus).

Where the oracle's sequential implicit Euler is affordable the whole trajectory is compared (1e-10
relative in the discrete L2 norm over all time points); otherwise its first steps are compared one
by one and, at sampled later steps, the step equations (M + kappa dt K) u_{k+1} = M u_k + dt F are
checked with the oracle's own matrices (a property that holds at any size)."""
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


def solver(insts, m, precision, tol, ctol=0.0):
    probs = [pm.problem(d["p"], d["n"], d["Nt"], d["kappa"], d["T"], d["domain"]) for d in insts]
    S = pm.Solver(probs, pm.default_mgrit_opts(cfactor=m, max_levels=12, coarsest_max=8, tol=tol),
                  pm.default_solver_opts(precision=precision, coarse_tol=ctol), device=0)
    for i, d in enumerate(insts):
        S.set_source(i, d["src"], d["tkind"])
    return S


def oracle_steps(d, nsteps):
    P = O.Problem(d["p"], d["n"], d["domain"])
    T = d["T"] * nsteps / d["Nt"]
    return P.sequential(d["kappa"], T, nsteps, P.load_vector(d["src"]), d["tkind"], np.zeros(P.ndof))


def step_residuals(d, U, ks):
    """max over sampled k of ||(M + kappa dt K) u_{k+1} - M u_k - dt F|| / ||M u_k + dt F|| (oracle matrices)"""
    P = O.Problem(d["p"], d["n"], d["domain"])
    M, K = P.scipy("M"), P.scipy("K")
    F = P.load_vector(d["src"])
    dt = d["T"] / d["Nt"]
    worst = 0.0
    for k in ks:
        b = M @ U[k] + dt * F
        r = (M + d["kappa"] * dt * K) @ U[k + 1] - b
        worst = max(worst, float(np.linalg.norm(r) / np.linalg.norm(b)))
    return worst


def test_mixed_precision_full_size(torch):
    cfg = W.config("heat-p4-h128-Nt2048")
    d = cfg["instances"][0]
    say("case full size p=4 h=2^-7 N_t=2048: FP64 and FP32-refined MGRIT")
    res = {}
    for prec in (0, 1):
        S = solver(cfg["instances"], cfg["m"], prec, 1e-10)
        (U,), st = S.solve_mgrit()
        res[prec] = U.cpu().numpy()
        say(f"  precision {prec}: iters {st['mgrit_iters']} V-cycles {st['vcycles']} t={st['t_solve_s']:.2f}s "
            f"levels {S.dims(0)[2]}")
        S.close()
    # FP32 V-cycle inside FP64 refinement: per-step error against the FP64 run
    per_step = np.linalg.norm(res[1] - res[0], axis=1) / np.maximum(np.linalg.norm(res[0], axis=1), 1e-300)
    say(f"  FP32-refined vs FP64: max per-step rel {per_step[1:].max():.2e}, total {rel(res[1], res[0]):.2e}")
    assert per_step[1:].max() <= 1e-10
    ns = 128
    Us = oracle_steps(d, ns)
    for prec in (0, 1):
        e = rel(res[prec][: ns + 1], Us)
        say(f"  precision {prec}: first {ns} steps vs oracle {e:.2e}")
        assert e <= EPS
        w = step_residuals(d, res[prec], [ns, 511, 1024, 1536, 2047])
        say(f"  precision {prec}: sampled step residuals {w:.2e}")
        assert w <= 1e-8


def test_heterogeneous_batch_full_size(torch):
    cfg = W.config("hetero-16")
    insts = cfg["instances"]
    say("case full size heterogeneous batch of 16 (FP32-refined, coarse tolerance 1e-6)")
    S = solver(insts, cfg["m"], 1, 1e-11, 1e-6)
    U, st = S.solve_mgrit()
    say(f"  iters {st['mgrit_iters']} V-cycles {st['vcycles']} t={st['t_solve_s']:.1f}s "
        f"groups {S.group_info(0)['groups']}")
    U = [u.cpu().numpy() for u in U]
    S.close()
    checked_full = checked_res = 0
    done128 = False
    for i, d in enumerate(insts):
        if d["n"] <= 64 or (d["n"] == 128 and not done128):
            done128 = done128 or d["n"] == 128
            e = rel(U[i], oracle_steps(d, d["Nt"]))
            say(f"  instance {i} p={d['p']} n={d['n']} domain={d['domain']}: eps={e:.2e}")
            assert e <= EPS
            checked_full += 1
    largest = max(range(len(insts)), key=lambda i: (insts[i]["n"], insts[i]["p"]))
    d = insts[largest]
    w = step_residuals(d, U[largest], [0, 100, 513, 1023])
    say(f"  instance {largest} p={d['p']} n={d['n']}: sampled step residuals {w:.2e}")
    assert w <= 1e-8
    checked_res += 1
    assert checked_full >= 9
