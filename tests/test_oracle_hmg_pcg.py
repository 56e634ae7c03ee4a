"""Pins of the oracle's p = 1 h-multigrid W-cycle and of its Jacobi-preconditioned CG (Sec. 4).

h-multigrid (the paper's p = 1 solve: one W-cycle, Gauss-Seidel smoothing, canonical prolongation,
weighted restriction, direct solve at the coarsest level):
- the prolongation writes a coarse degree-1 spline in the fine basis: both coefficient vectors
  describe the same function (checked by evaluating the two splines);
- on the square the Galerkin coarse operator equals the degree-1 matrices assembled on the coarse
  mesh (nested spaces, exact integration);
- nodes of one Gauss-Seidel colour never couple, and a sweep is the exact block update of each
  colour in turn;
- a mesh with at most 4 elements per direction is solved directly (one cycle is exact); on finer
  meshes the W-cycle contracts the error by a factor bounded independently of h.
CG: converges to the dense solution; its first iterate is the preconditioned steepest-descent
step; on a tiny system it terminates within n iterations.
"""
import numpy as np
import pytest

import oracle as O


def test_hmg_levels():
    assert O.Problem(2, 64, 0).hmg_levels() == [64, 32, 16, 8, 4]
    assert O.Problem(2, 12, 0).hmg_levels() == [12, 6, 3]
    assert O.Problem(2, 9, 0).hmg_levels() == [9]
    assert O.Problem(3, 4, 0).hmg_levels() == [4]


@pytest.mark.parametrize("domain", [0, 1])
def test_prolongation_represents_the_coarse_function(domain):
    n = 8
    P = O.Problem(2, n, domain)
    Pk = P.hmg_matrix(1.0, 0.01, 1, "P")
    fine, coarse = O.Problem(1, n, domain), O.Problem(1, n // 2, domain)
    assert Pk.shape == (fine.ndof, coarse.ndof)
    rng = np.random.default_rng(4)
    c = rng.standard_normal(coarse.ndof)
    cf = Pk @ c
    for s, t in rng.uniform(0, 1, (25, 2)):
        assert fine.eval(cf, s, t) == pytest.approx(coarse.eval(c, s, t), abs=1e-13)


@pytest.mark.parametrize("n,theta", [(8, 1.0), (16, 0.5)])
def test_galerkin_coarse_operator_is_rediscretisation_on_square(n, theta):
    kappa, dt = 1.7, 0.02
    P = O.Problem(3, n, 0)
    A1 = P.hmg_matrix(kappa, dt, 1, "A", theta=theta).toarray()
    Q = O.Problem(1, n // 2, 0)
    Ae = Q.dense("M") + theta * kappa * dt * Q.dense("K")
    assert np.allclose(A1, Ae, rtol=1e-12, atol=1e-15)
    # and level 0 is the rediscretised degree-1 operator of the problem itself
    A0 = P.hmg_matrix(kappa, dt, 0, "A", theta=theta).toarray()
    assert np.allclose(A0, P.dense("M1") + theta * kappa * dt * P.dense("K1"), rtol=1e-14, atol=1e-16)


def test_gauss_seidel_colour_sweep():
    n, kappa, dt = 6, 1.0, 0.05
    P = O.Problem(2, n, 1)
    A = P.dense("M1") + kappa * dt * P.dense("K1")
    n1 = n - 1
    colour = np.array([(ix % 2) + 2 * (iy % 2) for iy in range(n1) for ix in range(n1)])
    rng = np.random.default_rng(8)
    b, x0 = rng.standard_normal(n1 * n1), rng.standard_normal(n1 * n1)
    for direction, order in ((1, [0, 1, 2, 3]), (-1, [3, 2, 1, 0])):
        x = x0.copy()
        for c in order:
            idx = np.where(colour == c)[0]
            Acc = A[np.ix_(idx, idx)]
            assert np.count_nonzero(Acc - np.diag(np.diag(Acc))) == 0  # one colour never couples
            rest = np.where(colour != c)[0]
            x[idx] = (b[idx] - A[np.ix_(idx, rest)] @ x[rest]) / np.diag(Acc)
        assert np.allclose(P.gs_sweep(kappa, dt, b, x0, direction), x, rtol=1e-13, atol=1e-14)


def test_wcycle_direct_on_coarsest_mesh():
    P = O.Problem(2, 4, 0)
    A = P.dense("M1") + 0.3 * P.dense("K1")
    b = np.random.default_rng(2).standard_normal(P.ndof1)
    x = P.hmg_cycles(1.0, 0.3, b, np.zeros(P.ndof1), 1)
    assert np.allclose(A @ x, b, atol=1e-13)


def _wcycle_rate(domain, n, kdt):
    P = O.Problem(2, n, domain)
    b = np.random.default_rng(n).standard_normal(P.ndof1)
    xe = P.hmg_cycles(1.0, kdt, b, np.zeros(P.ndof1), 60)
    if n <= 16:
        A = P.dense("M1") + kdt * P.dense("K1")
        assert np.allclose(A @ xe, b, rtol=1e-10, atol=1e-12)
    x5 = P.hmg_cycles(1.0, kdt, b, np.zeros(P.ndof1), 5)
    x6 = P.hmg_cycles(1.0, kdt, b, np.zeros(P.ndof1), 6)
    return np.linalg.norm(x6 - xe) / np.linalg.norm(x5 - xe)


def test_wcycle_contraction_is_h_independent():
    # error contraction per W-cycle with kappa dt / h^2 fixed (the stiffness-dominated regime the
    # coarse MGRIT levels reach): bounded independently of h.  On the square (isotropic) it is the
    # textbook ~0.18; the quarter annulus has cells of aspect ratio up to pi / 2 * 2, where point
    # Gauss-Seidel with standard coarsening is slower, but the factor still settles as h shrinks.
    sq = [_wcycle_rate(0, n, 0.01 * (64 / n) ** 2) for n in (8, 16, 32, 64, 128)]
    assert max(sq) < 0.2, sq
    an = [_wcycle_rate(1, n, 0.01 * (64 / n) ** 2) for n in (8, 16, 32, 64, 128)]
    assert max(an) < 0.7 and abs(an[-1] - an[-2]) < 0.03, an


@pytest.mark.parametrize("p,n,domain", [(2, 8, 0), (4, 8, 1), (3, 16, 0)])
def test_pmg_with_wcycle_matches_dense(p, n, domain):
    P = O.Problem(p, n, domain)
    kappa, dt = 1.3, 0.01
    A = P.dense("M") + kappa * dt * P.dense("K")
    b = np.random.default_rng(5).standard_normal(P.ndof)
    rc, x, cyc = P.pmg_solve(kappa, dt, b, coarse=1)
    rc0, x0, cyc0 = P.pmg_solve(kappa, dt, b, coarse=0)
    assert rc == 0 and 1 <= cyc <= cyc0 + 3
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b) * 1.0001
    assert np.linalg.norm(x - np.linalg.solve(A, b)) / np.linalg.norm(x) < 1e-9


@pytest.mark.parametrize("p,n,domain", [(2, 8, 0), (5, 6, 1)])
def test_pcg_matches_dense(p, n, domain):
    P = O.Problem(p, n, domain)
    kappa, dt = 0.8, 0.02
    A = P.dense("M") + kappa * dt * P.dense("K")
    b = np.random.default_rng(6).standard_normal(P.ndof)
    rc, x, it = P.pmg_solve(kappa, dt, b, solver=1, maxcyc=5000)
    assert rc == 0 and it >= 2
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b) * 1.0001
    assert np.linalg.norm(x - np.linalg.solve(A, b)) / np.linalg.norm(x) < 1e-9


def test_pcg_first_iterate_is_preconditioned_steepest_descent():
    P = O.Problem(3, 5, 1)
    kappa, dt = 1.0, 0.05
    A = P.dense("M") + kappa * dt * P.dense("K")
    b = np.random.default_rng(7).standard_normal(P.ndof)
    rc, x1, it = P.pmg_solve(kappa, dt, b, solver=1, maxcyc=1)
    assert rc == -5 and it == 1  # stopped by the iteration cap after one step
    z = b / np.diag(A)
    alpha = (b @ z) / (z @ A @ z)
    assert np.allclose(x1, alpha * z, rtol=1e-12, atol=1e-15)


def test_pcg_finite_termination():
    P = O.Problem(2, 4, 0)  # 16 unknowns
    A = P.dense("M") + 0.1 * P.dense("K")
    b = np.random.default_rng(3).standard_normal(P.ndof)
    rc, x, it = P.pmg_solve(1.0, 0.1, b, solver=1, tol=1e-13, maxcyc=P.ndof + 2)
    assert rc == 0 and it <= P.ndof + 1
    assert np.allclose(A @ x, b, atol=1e-12)


def test_pcg_needs_more_iterations_as_p_grows():
    # the p-dependence the paper's comparison is about: CG iterations grow with p, p-MG cycles do not
    its, cycs = [], []
    for p in (2, 3, 4, 5):
        P = O.Problem(p, 16, 0)
        b = np.random.default_rng(p).standard_normal(P.ndof)
        its.append(P.pmg_solve(1.0, 0.01, b, solver=1, maxcyc=10000)[2])
        cycs.append(P.pmg_solve(1.0, 0.01, b)[2])
    assert its == sorted(its) and its[-1] > 2 * its[0], its
    assert max(cycs) <= 2 * min(cycs) + 1, cycs
