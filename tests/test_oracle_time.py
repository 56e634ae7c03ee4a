"""Pins of the oracle's time stepping and MGRIT (Sec. 2 eq:los, Sec. 3).

- Sequential implicit Euler is the block forward solve of A u = g (eq:mgrit).
- Manufactured solution u = sin(pi x) sin(pi y) e^{-t}: the error with respect to the
  time-discrete closed form converges at order p+1 in h.
- Converged MGRIT reproduces sequential time stepping.
- With a single coarse interval the first FCF-relaxation is already exact.
- Two-level MGRIT (parareal property): after k iterations the C-points 1..2k+1 are exact.
- The iteration counts stay in the range printed in Tables 7 and 8.
"""
import os

import numpy as np
import pytest

import oracle as O


def c1_problem(p=2, n=16, kappa=1.0):
    P = O.Problem(p, n, 0)
    F = P.load_vector([(1, 1, 2 * np.pi ** 2 * kappa - 1)])
    u0 = P.project([(1, 1, 1.0)])
    return P, F, u0


def test_sequential_is_block_forward_solve():
    P, F, u0 = c1_problem(2, 6)
    kappa, T, Nt = 1.0, 0.1, 12
    U = P.sequential(kappa, T, Nt, F, 1, u0)
    M, K = P.dense("M"), P.dense("K")
    dt = T / Nt
    assert np.array_equal(U[0], u0)
    for k in range(Nt):
        res = (M + kappa * dt * K) @ U[k + 1] - M @ U[k] - dt * np.exp(-(k + 1) * dt) * F
        assert np.abs(res).max() < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3])
def test_manufactured_solution_order(p):
    kappa, T, Nt = 1.0, 0.1, 8
    dt = T / Nt
    # time-discrete closed form of implicit Euler for the exact spatial mode:
    # a_{k+1} (1 + 2 pi^2 kappa dt) = a_k + dt (2 pi^2 kappa - 1) e^{-t_{k+1}}
    a = [1.0]
    for k in range(Nt):
        a.append((a[-1] + dt * (2 * np.pi ** 2 * kappa - 1) * np.exp(-(k + 1) * dt)) / (1 + 2 * np.pi ** 2 * kappa * dt))
    errs = []
    for n in (4, 8, 16):
        P, F, u0 = c1_problem(p, n, kappa)
        U = P.sequential(kappa, T, Nt, F, 1, u0)
        errs.append(P.l2_error_sinsin(U[-1], a[-1]))
    rate = np.log2(errs[-2] / errs[-1])
    assert rate == pytest.approx(p + 1, abs=0.3), errs


def test_mgrit_two_level_matches_sequential_c1():
    P, F, u0 = c1_problem()
    kappa, T, Nt = 1.0, 0.1, 128
    Us = P.sequential(kappa, T, Nt, F, 1, u0)
    for guess in (0, 1, 2):
        r = P.mgrit(kappa, T, Nt, F, 1, u0, m=4, max_levels=2, tol=1e-10, guess=guess)
        assert r["rc"] == 0
        assert 3 <= r["iters"] <= 12
        eps = np.linalg.norm(r["U"] - Us) / np.linalg.norm(Us)
        assert eps < 1e-10, eps
        # relative residual history decreases to the tolerance
        assert r["hist"][-1] <= 1e-10 and r["hist"][0] == 1.0


def test_mgrit_multilevel_matches_sequential():
    P = O.Problem(3, 8, 0)
    modes = [(1, 2, 0.7), (3, 1, -1.1), (2, 2, 0.4)]
    F = P.load_vector(modes)
    u0 = np.zeros(P.ndof)
    kappa, T, Nt = 0.8, 0.1, 256
    Us = P.sequential(kappa, T, Nt, F, 0, u0)
    r = P.mgrit(kappa, T, Nt, F, 0, u0, m=4, coarsest_max=8, tol=1e-11)
    assert r["rc"] == 0
    eps = np.linalg.norm(r["U"] - Us) / np.linalg.norm(Us)
    assert eps < 1e-10, eps


def test_single_coarse_interval_exact_after_first_fcf():
    P, F, u0 = c1_problem(2, 6)
    kappa, T, Nt = 1.0, 0.1, 8
    Us = P.sequential(kappa, T, Nt, F, 1, u0)
    r = P.mgrit(kappa, T, Nt, F, 1, u0, m=Nt, max_levels=2, tol=1e-10, stol=1e-14)
    assert r["rc"] == 0 and r["iters"] == 0
    assert np.linalg.norm(r["U"] - Us) / np.linalg.norm(Us) < 1e-12


def test_two_level_finite_termination():
    # Exactness travels along the coarse grid: every FCF sweep makes two more C-points exact
    # (each F-sweep carries the exact C-point through one interval), and the coarse correction
    # in between keeps what is exact.  So after k iterations (k corrections, k+1 FCF sweeps)
    # the C-points j <= 2k+1 equal the sequential solution and point 2k+2 does not yet.
    P = O.Problem(2, 6, 0)
    F = P.load_vector([(1, 1, 30.0), (2, 3, -20.0)])
    u0 = P.project([(1, 2, 1.0), (3, 3, 0.5)])
    kappa, T, Nt, m = 1.0, 2.0, 32, 4
    Us = P.sequential(kappa, T, Nt, F, 1, u0)
    for k in (0, 1, 2, 3):
        r = P.mgrit(kappa, T, Nt, F, 1, u0, m=m, max_levels=2, tol=0.0, max_iter=k, stol=1e-14)
        assert r["rc"] == -6 and r["iters"] == k
        U = r["U"]
        err = [np.linalg.norm(U[j * m] - Us[j * m]) / np.linalg.norm(Us[j * m]) for j in range(1, Nt // m + 1)]
        for j in range(1, 2 * k + 2):
            assert err[j - 1] < 1e-12, (k, j, err)
        assert err[2 * k + 1] > 1e-9, (k, err)


def _table_rows():
    path = os.path.join(os.path.dirname(__file__), "golden", "table7_8_mgrit_iterations.txt")
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            t, dom, h, nt, *its = [c.strip() for c in line.split("|")]
            rows.append((int(t), dom, int(h.split("^-")[1]), int(nt), [int(v) for v in its]))
    return rows


@pytest.mark.slow
def test_iteration_counts_in_printed_range():
    # Table 8 setting (N_t = 100, h = 2^-6, f = 1, u0 = 0, kappa = 1, T = 0.1), p = 2, both
    # domains.  m and the level count are not printed; m = 4 down to <= 8 intervals is used.
    rows = [r for r in _table_rows() if r[0] == 8 and r[2] == 6]
    assert len(rows) == 2
    for (_, dom, hexp, nt, its) in rows:
        P = O.Problem(2, 2 ** hexp, 0 if dom == "square" else 1)
        F = P.load_vector([(0, 0, 1.0)])
        r = P.mgrit(1.0, 0.1, nt, F, 0, np.zeros(P.ndof), m=4, coarsest_max=8, tol=1e-10)
        assert r["rc"] == 0
        assert abs(r["iters"] - its[0]) <= 3, (dom, r["iters"], its[0])
