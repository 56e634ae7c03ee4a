"""Pins of the oracle's theta-scheme (Sec. 2, eq:los), its MGRIT cycle types (Sec. 3, V-, W- and
F-cycles), the FP32-refined variant and the threaded sweeps.

- A sequential theta step solves (M + theta kappa dt K) u_{k+1} = (M - (1 - theta) kappa dt K) u_k +
  dt f (block forward solve, checked with the dense matrices).
- Against the exact solution of the semi-discrete system M u' + kappa K u = f (eigen-decomposition
  of the pencil (K, M), closed form in time), backward and forward Euler converge at order 1 and
  Crank-Nicolson at order 2 in dt.
- Converged MGRIT reproduces sequential stepping for every theta, cycle type, precision and
  spatial solver; W-cycles need no more iterations than V-cycles; with two levels all cycle types
  coincide (the coarsest level is solved exactly).
- Threads over the independent intervals of a sweep change nothing (bitwise).
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O


def _setup(p=2, n=4, domain=0, seed=3):
    P = O.Problem(p, n, domain)
    rng = np.random.default_rng(seed)
    F = P.load_vector([(1, 1, 1.0), (2, 1, -0.5)])
    u0 = P.project([(1, 2, 0.7)])
    return P, F, u0, rng


@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_theta_step_is_block_forward_solve(theta):
    P, F, u0, _ = _setup(2, 5, 1)
    kappa, T, Nt = 0.9, 0.01, 6
    U = P.sequential(kappa, T, Nt, F, 1, u0, theta=theta)
    M, K = P.dense("M"), P.dense("K")
    dt = T / Nt
    for k in range(Nt):
        w = dt * (theta * np.exp(-(k + 1) * dt) + (1 - theta) * np.exp(-k * dt))
        res = (M + theta * kappa * dt * K) @ U[k + 1] - (M - (1 - theta) * kappa * dt * K) @ U[k] - w * F
        assert np.abs(res).max() < 1e-13


def _semidiscrete_exact(P, kappa, T, F, u0):
    M, K = P.dense("M"), P.dense("K")
    lam, V = sl.eigh(K, M)  # V^T M V = I, K V = M V diag(lam)
    a0 = V.T @ M @ u0
    fh = V.T @ F
    e = np.exp(-kappa * lam * T)
    return V @ (a0 * e + fh * (1 - e) / (kappa * lam)), lam.max()


@pytest.mark.parametrize("theta,order", [(1.0, 1), (0.5, 2), (0.0, 1)])
def test_theta_scheme_time_order(theta, order):
    P, F, u0, _ = _setup(2, 3, 0)
    kappa, T = 1.0, 0.05
    ue, lmax = _semidiscrete_exact(P, kappa, T, F, u0)
    # forward Euler is stable for dt kappa lambda_max <= 2: start from a step count that keeps it
    # well inside
    N0 = max(16, int(2 ** np.ceil(np.log2(kappa * lmax * T))))
    errs = []
    for Nt in (N0, 2 * N0, 4 * N0):
        U = P.sequential(kappa, T, Nt, F, 0, u0, theta=theta)
        errs.append(np.linalg.norm(U[-1] - ue))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[-1] == pytest.approx(order, abs=0.15), (errs, rates)


@pytest.mark.parametrize("theta", [0.5, 1.0])
@pytest.mark.parametrize("cycle", [0, 1, 2])
def test_mgrit_theta_and_cycles_match_sequential(theta, cycle):
    P, F, u0, _ = _setup(3, 6, 1)
    kappa, T, Nt = 1.0, 0.1, 64
    Us = P.sequential(kappa, T, Nt, F, 0, u0, theta=theta)
    r = P.mgrit(kappa, T, Nt, F, 0, u0, m=4, coarsest_max=2, tol=1e-12, theta=theta, cycle=cycle, stol=1e-13)
    assert r["rc"] == 0
    assert np.linalg.norm(r["U"] - Us) / np.linalg.norm(Us) < 1e-10


def test_forward_euler_mgrit_matches_sequential():
    # explicit steps on every level: the hierarchy is kept shallow enough that dt_l kappa lambda_max
    # stays below 2 on the coarsest level
    P, F, u0, _ = _setup(2, 3, 0)
    kappa, T = 1.0, 0.05
    _, lmax = _semidiscrete_exact(P, kappa, T, F, u0)
    Nt = int(2 ** np.ceil(np.log2(4 * kappa * lmax * T * 2)))
    Us = P.sequential(kappa, T, Nt, F, 0, u0, theta=0.0)
    r = P.mgrit(kappa, T, Nt, F, 0, u0, m=2, max_levels=3, coarsest_max=1, tol=1e-12, theta=0.0, stol=1e-13)
    assert r["rc"] == 0
    assert np.linalg.norm(r["U"] - Us) / np.linalg.norm(Us) < 1e-10


def test_w_cycle_needs_no_more_iterations():
    P, F, u0, _ = _setup(2, 8, 0)
    kappa, T, Nt = 1.0, 0.1, 256
    it = {}
    for cycle in (0, 1, 2):
        r = P.mgrit(kappa, T, Nt, F, 0, u0, m=4, coarsest_max=4, tol=1e-10, cycle=cycle)
        assert r["rc"] == 0
        it[cycle] = r["iters"]
    assert it[1] <= it[0] and it[2] <= it[0], it


def test_two_level_cycles_coincide():
    P, F, u0, _ = _setup(2, 6, 0)
    res = [P.mgrit(1.0, 0.1, 32, F, 0, u0, m=4, max_levels=2, tol=1e-10, cycle=c) for c in (0, 1, 2)]
    for r in res[1:]:
        assert r["iters"] == res[0]["iters"] and np.array_equal(r["U"], res[0]["U"])


@pytest.mark.parametrize("prec,coarse,solver", [(1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1)])
def test_mgrit_solver_variants_match_sequential(prec, coarse, solver):
    P, F, u0, _ = _setup(3, 8, 1)
    kappa, T, Nt = 0.5, 0.1, 64
    Us = P.sequential(kappa, T, Nt, F, 0, u0)
    r = P.mgrit(kappa, T, Nt, F, 0, u0, m=4, coarsest_max=4, tol=1e-12, stol=1e-13, prec=prec, coarse=coarse,
                solver=solver, maxcyc=5000)
    assert r["rc"] == 0
    assert np.linalg.norm(r["U"] - Us) / np.linalg.norm(Us) < 1e-10


def test_threads_change_nothing():
    P, F, u0, _ = _setup(3, 8, 0)
    a = P.mgrit(1.0, 0.1, 128, F, 0, u0, m=4, coarsest_max=4, tol=1e-10, threads=1)
    b = P.mgrit(1.0, 0.1, 128, F, 0, u0, m=4, coarsest_max=4, tol=1e-10, threads=4)
    assert a["iters"] == b["iters"] and a["cycles"] == b["cycles"] and a["solves"] == b["solves"]
    assert np.array_equal(a["U"], b["U"]) and np.array_equal(a["hist"], b["hist"])
