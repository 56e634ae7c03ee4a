"""Pins of the oracle's geometry, assembly and transfer operators.

- Mass matrix entries of the full space sum to the area of Omega (square 1, quarter annulus
  3 pi / 4); the stiffness matrix annihilates constants (Sec. 2, eq:los).
- At p = 1 the discretisation is the textbook bilinear finite-element one.
- L2-projection transfers with row-sum lumping preserve constants (Sec. 4, eq:prolongation, eq:PM).
- The L2 projection of sin(pi x) sin(pi y) converges at order p+1.
"""
import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("p,n", [(1, 4), (2, 5), (3, 4), (5, 3)])
def test_square_mass_sum_and_stiffness_null(p, n):
    P = O.Problem(p, n, 0)
    M = P.dense("Mfull")
    K = P.dense("Kfull")
    assert M.sum() == pytest.approx(1.0, rel=1e-13)
    assert np.abs(K @ np.ones(K.shape[0])).max() < 1e-12
    assert np.abs(M - M.T).max() < 1e-15 and np.abs(K - K.T).max() < 1e-14
    Mr, Kr = P.dense("M"), P.dense("K")
    assert np.linalg.eigvalsh(Mr).min() > 0 and np.linalg.eigvalsh(Kr).min() > 0
    assert Mr.shape == ((n + p - 2) ** 2,) * 2


@pytest.mark.parametrize("p", [2, 3])
def test_annulus_area_and_geometry(p):
    P = O.Problem(p, 16, 1)
    M = P.dense("Mfull")
    # quadrature of the rational Jacobian is not exact: error far below the mesh scale
    assert M.sum() == pytest.approx(3 * np.pi / 4, rel=1e-8)
    K = P.dense("Kfull")
    assert np.abs(K @ np.ones(K.shape[0])).max() < 1e-11
    # the map: inner arc r = 1 at s = 0, outer r = 2 at s = 1; angle 0 at t = 0, pi/2 at t = 1
    for s in (0.0, 0.3, 1.0):
        for t in (0.0, 0.25, 0.5, 0.9, 1.0):
            X, J = O.geom(1, s, t)
            assert np.hypot(*X) == pytest.approx(1.0 + s, rel=1e-14)
            h = 1e-6
            if 0 < s < 1 and 0 < t < 1:
                Xs = (O.geom(1, s + h, t)[0] - O.geom(1, s - h, t)[0]) / (2 * h)
                Xt = (O.geom(1, s, t + h)[0] - O.geom(1, s, t - h)[0]) / (2 * h)
                assert np.allclose(J[:, 0], Xs, atol=1e-8) and np.allclose(J[:, 1], Xt, atol=1e-8)
    assert np.allclose(O.geom(1, 0, 0)[0], [1, 0]) and np.allclose(O.geom(1, 0, 1)[0], [0, 1], atol=1e-15)


@pytest.mark.parametrize("n", [3, 6])
def test_p1_is_bilinear_fem(n):
    P = O.Problem(1, n, 0)
    h = 1.0 / n
    m = n - 1
    M1 = (h / 6) * (4 * np.eye(m) + np.eye(m, k=1) + np.eye(m, k=-1))
    K1 = (1 / h) * (2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1))
    assert np.allclose(P.dense("M"), np.kron(M1, M1), atol=1e-15)
    assert np.allclose(P.dense("K"), np.kron(K1, M1) + np.kron(M1, K1), atol=1e-13)
    # the degree-1 matrices of any degree-p problem are the same objects
    Pp = O.Problem(3, n, 0)
    assert np.allclose(Pp.dense("M1"), np.kron(M1, M1), atol=1e-15)
    assert np.allclose(Pp.dense("K1"), np.kron(K1, M1) + np.kron(M1, K1), atol=1e-13)


@pytest.mark.parametrize("p,domain", [(2, 0), (4, 0), (3, 1)])
def test_transfer_preserves_constants(p, domain):
    n = 6
    P = O.Problem(p, n, domain)
    Pf = P.dense("Pfull")
    Mf, M1f = P.dense("Mfull"), P.dense("M1full")
    mlp_full, ml1_full = Mf.sum(1), M1f.sum(1)
    # partition of unity of both bases: row sums of P_1^p are the degree-p lumped masses,
    # column sums the degree-1 lumped masses
    assert np.allclose(Pf.sum(1), mlp_full, rtol=1e-12, atol=1e-15)
    assert np.allclose(Pf.sum(0), ml1_full, rtol=1e-12, atol=1e-15)
    # both transfer operators of eq:prolongation map the constant to the constant on the full spaces
    assert np.allclose((Pf @ np.ones(Pf.shape[1])) / mlp_full, 1.0, rtol=1e-12)
    assert np.allclose((Pf.T @ np.ones(Pf.shape[0])) / ml1_full, 1.0, rtol=1e-12)
    # the interior lumped masses returned are the full-row sums restricted to the interior
    mlp, ml1 = P.lumped()
    N, N1 = n + p, n + 1
    inner = [iy * N + ix for iy in range(1, N - 1) for ix in range(1, N - 1)]
    inner1 = [iy * N1 + ix for iy in range(1, N1 - 1) for ix in range(1, N1 - 1)]
    assert np.allclose(mlp, mlp_full[inner], rtol=1e-15)
    assert np.allclose(ml1, ml1_full[inner1], rtol=1e-15)
    # and the interior P is the interior block of the full one
    assert np.allclose(P.dense("P"), Pf[np.ix_(inner, inner1)])


def test_constant_source_load_vector():
    # f = 1 is the mode (0,0,1): int Phi_i = lumped mass (partition of unity)
    P = O.Problem(3, 6, 1)
    mlp, _ = P.lumped()
    assert np.allclose(P.load_vector([(0, 0, 1.0)]), mlp, rtol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_projection_converges_at_order_p_plus_1(p):
    errs = []
    ns = [4, 8, 16]
    for n in ns:
        P = O.Problem(p, n, 0)
        c = P.project([(1, 1, 1.0)])
        errs.append(P.l2_error_sinsin(c, 1.0))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    assert rates[-1] == pytest.approx(p + 1, abs=0.25), (errs, rates)


def _ann_u(x, y):
    r2 = x * x + y * y
    return (r2 - 1.0) * (4.0 - r2) * x * y


def _ann_f(x, y):
    # -Laplace of _ann_u, worked out by hand: u = g(rho) x y with rho = x^2 + y^2 and
    # g = -rho^2 + 5 rho - 4, so Lap u = x y (Lap g) + 2 grad g . grad(x y) = x y (60 - 32 rho)
    return x * y * (32.0 * (x * x + y * y) - 60.0)


def test_annulus_manufactured_laplacian_is_right():
    # the hand-derived source really is -Lap u (second differences at a few points)
    h = 1e-4
    for x, y in [(1.2, 0.3), (0.5, 1.4), (1.0, 1.0)]:
        lap = (_ann_u(x + h, y) + _ann_u(x - h, y) + _ann_u(x, y + h) + _ann_u(x, y - h) - 4 * _ann_u(x, y)) / h ** 2
        assert -lap == pytest.approx(_ann_f(x, y), rel=1e-5)


@pytest.mark.parametrize("p", [2, 3])
def test_annulus_stiffness_manufactured_convergence(p):
    # u = (x^2 + y^2 - 1)(4 - x^2 - y^2) x y vanishes on all four sides of the quarter annulus
    # (r = 1, r = 2, x = 0, y = 0); the IgA solution of K c = int f Phi with f = -Lap u must converge
    # to it at order p + 1 in L2.  Any error in the mapped gradients (e.g. J^{-1} in place of J^{-T})
    # or in the geometry breaks the rate.
    errs = []
    for n in (4, 8, 16):
        P = O.Problem(p, n, 1)
        c = np.linalg.solve(P.dense("K"), P.load_vector_fn(_ann_f))
        errs.append(P.l2_error_fn(c, _ann_u))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] == pytest.approx(p + 1, abs=0.3), (errs, rates)


def test_load_vector_fn_matches_modes_on_square():
    # on the unit square physical and parameter coordinates agree, so a function source equals the
    # modal source with the same terms
    P = O.Problem(3, 6, 0)
    f = lambda x, y: 0.7 * np.sin(2 * np.pi * x) * np.sin(np.pi * y) - 1.3
    assert np.allclose(P.load_vector_fn(f), P.load_vector([(2, 1, 0.7), (0, 0, -1.3)]), rtol=1e-12, atol=1e-15)
