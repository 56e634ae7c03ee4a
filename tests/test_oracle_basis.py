"""Pins of the oracle's B-spline basis and quadrature against what the paper and mathematics fix.

- Fig. 1 (Sec. 2): the printed piecewise linear and quadratic basis functions.
- Sec. 2: partition of unity, interpolation at both ends of an open knot vector.
- Textbook closed forms: int phi_{i,p} = (xi_{i+p+1} - xi_i) / (p+1); Gauss-Legendre exactness.
"""
import ast
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig1_bspline_pieces.txt")

_ALLOWED = (ast.Expression, ast.BinOp, ast.UnaryOp, ast.Constant, ast.Name, ast.Load, ast.Add, ast.Sub,
            ast.Mult, ast.Div, ast.USub, ast.UAdd)


def _safe_poly(expr: str):
    tree = ast.parse(expr, mode="eval")
    for node in ast.walk(tree):
        if not isinstance(node, _ALLOWED) or (isinstance(node, ast.Name) and node.id != "x"):
            raise ValueError(f"unexpected token in golden expression: {expr}")
    code = compile(tree, "<golden>", "eval")
    return lambda x: eval(code, {"__builtins__": {}}, {"x": x})


def _pieces():
    out = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        deg, kn, idx, lo, hi, ex = [c.strip() for c in line.split("|")]
        out.append((int(deg), [float(v) for v in kn.split(",")], int(idx), float(lo), float(hi), _safe_poly(ex)))
    return out


def test_fig1_printed_pieces():
    pieces = _pieces()
    assert len(pieces) == 15
    xs = np.linspace(0.0, 3.0, 61)[:-1] + 0.013  # points inside the knot spans
    for deg in (1, 2):
        sel = [p for p in pieces if p[0] == deg]
        kn = sel[0][1]
        nfun = len(kn) - deg - 1
        for i in range(nfun):
            mine = [p for p in sel if p[2] == i]
            for x in xs:
                want = 0.0
                for (_, _, _, lo, hi, f) in mine:
                    if lo <= x < hi:
                        want = f(x)
                got = O.bspline(kn, i, deg, x)
                assert got == pytest.approx(want, abs=1e-14), (deg, i, x)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_partition_of_unity_and_ends(p):
    n = 7
    xi = O.knots(p, n)
    N = n + p
    assert len(xi) == n + 2 * p + 1
    for x in np.linspace(0, 1, 97):
        vals = np.array([O.bspline(xi, i, p, x) for i in range(N)])
        assert vals.sum() == pytest.approx(1.0, abs=1e-14)
        assert vals.min() >= -1e-15
    # interpolatory at both ends: only the first / last function is non-zero there
    v0 = np.array([O.bspline(xi, i, p, 0.0) for i in range(N)])
    v1 = np.array([O.bspline(xi, i, p, 1.0) for i in range(N)])
    assert v0[0] == 1.0 and np.all(v0[1:] == 0.0)
    assert v1[-1] == 1.0 and np.all(v1[:-1] == 0.0)


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_integral_closed_form(p):
    n = 5
    xi = O.knots(p, n)
    gx, gw = O.gauss(p + 1)
    for i in range(n + p):
        s = 0.0
        for e in range(n):
            a, b = e / n, (e + 1) / n
            for x, w in zip(gx, gw):
                s += w * (b - a) * O.bspline(xi, i, p, a + (b - a) * x)
        assert s == pytest.approx((xi[i + p + 1] - xi[i]) / (p + 1), rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("p", [1, 2, 4])
def test_derivative_vs_difference(p):
    xi = O.knots(p, 6)
    rng = np.random.default_rng(1)
    for x in rng.uniform(0.01, 0.99, 25):
        for i in range(6 + p):
            h = 1e-6
            fd = (O.bspline(xi, i, p, x + h) - O.bspline(xi, i, p, x - h)) / (2 * h)
            # skip points within h of a knot, where the derivative may jump
            if np.min(np.abs(xi - x)) < 2 * h:
                continue
            assert O.bspline(xi, i, p, x, deriv=True) == pytest.approx(fd, abs=1e-6)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 6, 8])
def test_gauss_exactness(q):
    x, w = O.gauss(q)
    assert np.all(np.diff(x) > 0) and x[0] > 0 and x[-1] < 1
    for d in range(2 * q):
        assert np.dot(w, x ** d) == pytest.approx(1.0 / (d + 1), rel=1e-13)
    # and not exact one degree higher (pins the number of points)
    d = 2 * q
    assert abs(np.dot(w, x ** d) - 1.0 / (d + 1)) > 1e-12
