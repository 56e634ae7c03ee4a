"""Pins of the oracle's direct solver, ILUT and p-multigrid (Sec. 4).

- The banded Cholesky solve equals a dense LAPACK solve.
- ILUT with tau = 0 and unlimited fill is the exact LU factorisation (unique without pivoting).
- ILUT respects its per-row caps and its drop rule.
- p-multigrid converges to the dense solution; with an exact smoother it needs one cycle.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O


def _dense_lu_nopivot(A):
    """Textbook Doolittle LU without pivoting (unit lower L)."""
    n = A.shape[0]
    L = np.eye(n)
    U = np.zeros_like(A)
    for i in range(n):
        for j in range(i, n):
            U[i, j] = A[i, j] - L[i, :i] @ U[:i, j]
        for j in range(i + 1, n):
            L[j, i] = (A[j, i] - L[j, :i] @ U[:i, i]) / U[i, i]
    return L, U


@pytest.mark.parametrize("p,n,domain", [(2, 6, 0), (3, 5, 1)])
def test_direct_solve_matches_lapack(p, n, domain):
    P = O.Problem(p, n, domain)
    c = 0.37
    A = P.dense("M") + c * P.dense("K")
    b = np.random.default_rng(3).standard_normal(P.ndof)
    x = P.direct_solve(c, b)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("p,n", [(2, 5), (3, 4)])
def test_ilut_exact_limit_is_lu(p, n):
    P = O.Problem(p, n, 0)
    c = 0.05
    A = P.dense("M") + c * P.dense("K")
    rc, L, U = P.ilut(c, tau=0.0, unlimited=True)
    assert rc == 0
    Le, Ue = _dense_lu_nopivot(A)
    assert np.allclose(L.toarray() + np.eye(P.ndof), Le, atol=1e-13)
    assert np.allclose(U.toarray(), Ue, rtol=1e-12, atol=1e-16)


def test_ilut_caps_and_structure():
    P = O.Problem(3, 8, 0)
    c = 1e-3
    A = (P.scipy("M") + c * P.scipy("K")).tocsr()
    rc, L, U = P.ilut(c, tau=1e-12)
    assert rc == 0
    Lc, Uc = L.tocoo(), U.tocoo()
    assert np.all(Lc.row > Lc.col) and np.all(Uc.row <= Uc.col)
    for i in range(P.ndof):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        assert L.indptr[i + 1] - L.indptr[i] <= np.sum(cols < i)
        assert U.indptr[i + 1] - U.indptr[i] - 1 <= np.sum(cols > i)
        assert U[i, i] > 0
    # caps bind: the factor is incomplete, but a close approximation of A
    E = (sp.eye(P.ndof) + L) @ U - A
    assert abs(E).max() > 0
    assert abs(E).max() < 1e-2 * abs(A).max()


def test_ilut_drop_rule_extreme():
    # a drop tolerance far above every ratio |w_j| / ||a_i|| keeps only the diagonal: U = diag(A)
    P = O.Problem(2, 5, 0)
    c = 0.1
    A = P.dense("M") + c * P.dense("K")
    rc, L, U = P.ilut(c, tau=10.0)
    assert rc == 0 and L.nnz == 0
    assert np.allclose(U.toarray(), np.diag(np.diag(A)))


@pytest.mark.parametrize("p,n,domain", [(2, 8, 0), (3, 8, 0), (4, 6, 1)])
def test_pmg_matches_dense_solve(p, n, domain):
    P = O.Problem(p, n, domain)
    kappa, dt = 1.3, 0.01
    A = P.dense("M") + kappa * dt * P.dense("K")
    b = np.random.default_rng(5).standard_normal(P.ndof)
    rc, x, cyc = P.pmg_solve(kappa, dt, b)
    assert rc == 0 and 1 <= cyc < 20
    xe = np.linalg.solve(A, b)
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b) * 1.0001
    assert np.linalg.norm(x - xe) / np.linalg.norm(xe) < 1e-9


def test_pmg_exact_smoother_one_cycle():
    # with tau = 0 and no per-row caps ILUT is the exact LU factorisation, so the first smoothing step
    # already solves the system and one V-cycle meets the tolerance
    P = O.Problem(2, 4, 0)
    b = np.random.default_rng(9).standard_normal(P.ndof)
    A = P.dense("M") + 0.02 * P.dense("K")
    for coarse in (0, 1):
        rc, x, cyc = P.pmg_solve(1.0, 0.02, b, tau=0.0, maxcyc=5, unlimited=True, coarse=coarse)
        assert rc == 0 and cyc == 1
        assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    # with the caps of A's pattern the factor is incomplete and needs more than one cycle
    rc, x, cyc = P.pmg_solve(1.0, 0.02, b, tau=0.0, maxcyc=50)
    assert rc == 0 and cyc > 1


@pytest.mark.parametrize("prec,coarse,solver", [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1)])
def test_sequential_iterative_matches_direct(prec, coarse, solver):
    # sequential stepping with any of the iterative spatial solvers reaches the direct solution of
    # every step (spatial tolerance 1e-13)
    P = O.Problem(3, 8, 1)
    F = P.load_vector([(1, 2, 0.8), (3, 1, -0.4)])
    u0 = P.project([(1, 1, 1.0)])
    Us = P.sequential(0.7, 0.1, 12, F, 0, u0)
    rc, U, cyc = P.sequential_pmg(0.7, 0.1, 12, F, 0, u0, stol=1e-13, maxcyc=2000, prec=prec, coarse=coarse,
                                  solver=solver)
    assert rc == 0 and cyc >= 12
    per = np.linalg.norm(U - Us, axis=1) / np.maximum(np.linalg.norm(Us, axis=1), 1e-300)
    assert per.max() <= 1e-11


@pytest.mark.parametrize("p,n,domain", [(2, 8, 0), (4, 6, 1)])
def test_pmg_fp32_refined_matches_dense(p, n, domain):
    # FP32 V-cycles inside FP64 refinement still reach the FP64 tolerance; the FP32 V-cycle contracts
    # about as well as the FP64 one, so the cycle counts stay close
    P = O.Problem(p, n, domain)
    kappa, dt = 1.3, 0.01
    A = P.dense("M") + kappa * dt * P.dense("K")
    b = np.random.default_rng(15).standard_normal(P.ndof)
    rc, x, cyc = P.pmg_solve(kappa, dt, b, prec=1)
    rc64, x64, cyc64 = P.pmg_solve(kappa, dt, b)
    assert rc == 0 and rc64 == 0
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b) * 1.0001
    assert abs(cyc - cyc64) <= 2


def test_coarse_correction_helps():
    # the p=1 correction must speed up plain ILUT iteration: compare the V-cycle count to a
    # pure smoothing iteration x += S (b - A x) run by hand from the oracle's factor
    P = O.Problem(2, 16, 0)
    kappa, dt = 1.0, 0.05
    A = P.scipy("M") + kappa * dt * P.scipy("K")
    b = np.random.default_rng(11).standard_normal(P.ndof)
    rc, x, cyc = P.pmg_solve(kappa, dt, b, tol=1e-10)
    assert rc == 0
    _, L, U = P.ilut(kappa * dt, tau=1e-12)
    Ls = (sp.eye(P.ndof) + L).tocsr()
    from scipy.sparse.linalg import spsolve_triangular
    y = np.zeros(P.ndof)
    k = 0
    while np.linalg.norm(b - A @ y) > 1e-10 * np.linalg.norm(b) and k < 200:
        r = b - A @ y
        z = spsolve_triangular(Ls, r, lower=True)
        y = y + spsolve_triangular(U.tocsr(), z, lower=False)
        k += 1
    assert 2 * cyc < k
