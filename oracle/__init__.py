"""Plain FP64 CPU oracle for MGRIT + p-multigrid on isogeometric heat equations.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline leg of the
benchmark are the only users.  The arithmetic lives in ``oracle.c`` (plain C, FP64, written
from the paper's definitions); this module only marshals numpy arrays through ctypes.  It
shares no code with the GPU library and never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_llp = C.POINTER(C.c_longlong)
FN2 = C.CFUNCTYPE(C.c_double, C.c_double, C.c_double)  # a function of the physical coordinates (x, y)


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_knots.argtypes = [C.c_int, C.c_int, _dp]
        L.orc_bspline.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_bspline.restype = C.c_double
        L.orc_bspline_deriv.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_bspline_deriv.restype = C.c_double
        L.orc_gauss.argtypes = [C.c_int, _dp, _dp]
        L.orc_geom.argtypes = [C.c_int, C.c_double, C.c_double, _dp]
        L.orc_problem_create.argtypes = [C.c_int, C.c_int, C.c_int]
        L.orc_problem_create.restype = C.c_void_p
        L.orc_problem_free.argtypes = [C.c_void_p]
        L.orc_problem_dims.argtypes = [C.c_void_p, _ip]
        L.orc_matrix_shape.argtypes = [C.c_void_p, C.c_int, _ip]
        L.orc_matrix_get.argtypes = [C.c_void_p, C.c_int, _ip, _ip, _dp]
        L.orc_lumped.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_load_vector.argtypes = [C.c_void_p, C.c_int, _ip, _ip, _dp, _dp]
        L.orc_eval_spline.argtypes = [C.c_void_p, _dp, C.c_double, C.c_double]
        L.orc_eval_spline.restype = C.c_double
        L.orc_l2_error_sinsin.argtypes = [C.c_void_p, _dp, C.c_double]
        L.orc_l2_error_sinsin.restype = C.c_double
        L.orc_direct_solve.argtypes = [C.c_void_p, C.c_double, _dp, _dp]
        L.orc_project.argtypes = [C.c_void_p, C.c_int, _ip, _ip, _dp, _dp]
        L.orc_ilut.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, _ip]
        L.orc_ilut_get.argtypes = [_ip, _ip, _dp, _ip, _ip, _dp]
        L.orc_pmg_solve.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                    C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, _ip]
        L.orc_sequential.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, _dp, C.c_int, _dp, _dp]
        L.orc_sequential_theta.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, _dp, C.c_int, C.c_double,
                                           _dp, _dp]
        L.orc_sequential_pmg.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, _dp, C.c_int, C.c_double, _dp,
                                         C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _llp]
        L.orc_mgrit.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, _dp, C.c_int, _dp, _ip, _dp, _dp, _ip,
                                _llp, _llp, _dp]
        L.orc_load_vector_fn.argtypes = [C.c_void_p, FN2, _dp]
        L.orc_l2_error_fn.argtypes = [C.c_void_p, _dp, FN2]
        L.orc_l2_error_fn.restype = C.c_double
        L.orc_hmg_info.argtypes = [C.c_void_p, _ip]
        L.orc_hmg_matrix.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, _ip, _ip, _ip,
                                     _dp]
        L.orc_hmg_cycles.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int, _dp, _dp]
        L.orc_gs_sweep.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int, _dp, _dp]
        L.orc_gs_sweep.restype = None
        _lib = L
    return _lib


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _i(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_ip)


def knots(p: int, n: int) -> np.ndarray:
    xi = np.zeros(n + 2 * p + 1)
    lib().orc_knots(p, n, _d(xi))
    return xi


def bspline(xi, i: int, p: int, x: float, deriv: bool = False) -> float:
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    f = lib().orc_bspline_deriv if deriv else lib().orc_bspline
    return f(_d(xi), len(xi), i, p, float(x))


def gauss(q: int):
    x = np.zeros(q)
    w = np.zeros(q)
    lib().orc_gauss(q, _d(x), _d(w))
    return x, w


def geom(domain: int, s: float, t: float):
    out = np.zeros(6)
    lib().orc_geom(domain, s, t, _d(out))
    return out[:2].copy(), out[2:].reshape(2, 2).copy()


# matrix selectors of orc_matrix_get
MATS = {"M": 0, "K": 1, "Mfull": 2, "Kfull": 3, "M1": 4, "K1": 5, "M1full": 6, "K1full": 7,
        "P": 8, "Pfull": 9}


class Problem:
    """Discretisation of degree p on n x n elements; domain 0 = unit square, 1 = quarter annulus."""

    def __init__(self, p: int, n: int, domain: int = 0):
        self.p, self.n, self.domain = p, n, domain
        h = lib().orc_problem_create(p, n, domain)
        if not h:
            raise ValueError("bad problem parameters")
        self._h = C.c_void_p(h)
        d = np.zeros(5, dtype=np.int32)
        lib().orc_problem_dims(self._h, _i(d))
        self.N, self.Nin, self.ndof, self.N1in, self.ndof1 = (int(v) for v in d)

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().orc_problem_free(self._h)
                self._h = None
        except Exception:
            pass

    def matrix(self, name: str):
        """CSR arrays (rowptr, colidx, values, shape) of one assembled matrix."""
        which = MATS[name]
        sh = np.zeros(3, dtype=np.int32)
        lib().orc_matrix_shape(self._h, which, _i(sh))
        nr, nc, nnz = (int(v) for v in sh)
        rp = np.zeros(nr + 1, dtype=np.int32)
        ci = np.zeros(nnz, dtype=np.int32)
        v = np.zeros(nnz)
        lib().orc_matrix_get(self._h, which, _i(rp), _i(ci), _d(v))
        return rp, ci, v, (nr, nc)

    def dense(self, name: str) -> np.ndarray:
        rp, ci, v, (nr, nc) = self.matrix(name)
        A = np.zeros((nr, nc))
        for i in range(nr):
            A[i, ci[rp[i]:rp[i + 1]]] += v[rp[i]:rp[i + 1]]
        return A

    def scipy(self, name: str):
        import scipy.sparse as sp
        rp, ci, v, shape = self.matrix(name)
        return sp.csr_matrix((v, ci, rp), shape=shape)

    def lumped(self):
        mlp = np.zeros(self.ndof)
        ml1 = np.zeros(self.ndof1)
        lib().orc_lumped(self._h, _d(mlp), _d(ml1))
        return mlp, ml1

    def load_vector(self, modes) -> np.ndarray:
        """int f Phi_i for f = sum amp sin(k pi s) sin(l pi t); modes = [(k, l, amp), ...]."""
        k = np.array([m[0] for m in modes], dtype=np.int32)
        l_ = np.array([m[1] for m in modes], dtype=np.int32)
        a = np.array([m[2] for m in modes], dtype=np.float64)
        out = np.zeros(self.ndof)
        lib().orc_load_vector(self._h, len(modes), _i(k), _i(l_), _d(a), _d(out))
        return out

    def project(self, modes) -> np.ndarray:
        k = np.array([m[0] for m in modes], dtype=np.int32)
        l_ = np.array([m[1] for m in modes], dtype=np.int32)
        a = np.array([m[2] for m in modes], dtype=np.float64)
        out = np.zeros(self.ndof)
        rc = lib().orc_project(self._h, len(modes), _i(k), _i(l_), _d(a), _d(out))
        if rc:
            raise RuntimeError(f"projection failed: {rc}")
        return out

    def eval(self, c: np.ndarray, s: float, t: float) -> float:
        c = np.ascontiguousarray(c, dtype=np.float64)
        return lib().orc_eval_spline(self._h, _d(c), s, t)

    def l2_error_sinsin(self, c: np.ndarray, a: float) -> float:
        c = np.ascontiguousarray(c, dtype=np.float64)
        return lib().orc_l2_error_sinsin(self._h, _d(c), a)

    def direct_solve(self, c: float, b: np.ndarray) -> np.ndarray:
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.ndof)
        rc = lib().orc_direct_solve(self._h, c, _d(b), _d(x))
        if rc:
            raise RuntimeError(f"direct solve failed: {rc}")
        return x

    def ilut(self, c: float, tau: float = 1e-12, unlimited: bool = False):
        """ILUT of M + c K: returns (L, U) as scipy CSR; L strict lower (unit diagonal implied)."""
        import scipy.sparse as sp
        nn = np.zeros(2, dtype=np.int32)
        rc = lib().orc_ilut(self._h, c, tau, 1 if unlimited else 0, _i(nn))
        n = self.ndof
        Lrp = np.zeros(n + 1, dtype=np.int32)
        Lci = np.zeros(max(int(nn[0]), 1), dtype=np.int32)
        Lv = np.zeros(max(int(nn[0]), 1))
        Urp = np.zeros(n + 1, dtype=np.int32)
        Uci = np.zeros(int(nn[1]), dtype=np.int32)
        Uv = np.zeros(int(nn[1]))
        lib().orc_ilut_get(_i(Lrp), _i(Lci), _d(Lv), _i(Urp), _i(Uci), _d(Uv))
        L = sp.csr_matrix((Lv[:nn[0]], Lci[:nn[0]], Lrp), shape=(n, n))
        U = sp.csr_matrix((Uv, Uci, Urp), shape=(n, n))
        return rc, L, U

    def pmg_solve(self, kappa: float, dt: float, b: np.ndarray, x0=None, tau=1e-12, nu1=1, nu2=1,
                  tol=1e-12, maxcyc=100, theta=1.0, prec=0, coarse=0, solver=0, unlimited=False):
        """Spatial solve of (M + theta kappa dt K) x = b from x0.  solver 0: p-multigrid (prec 1: FP32
        V-cycle in FP64 refinement; coarse 0: exact p = 1 solve, 1: one h-multigrid W-cycle); solver 1:
        Jacobi-preconditioned CG.  unlimited: ILUT without per-row caps.  Returns (rc, x, cycles)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.ndof) if x0 is None else np.array(x0, dtype=np.float64)
        cyc = C.c_int(0)
        rc = lib().orc_pmg_solve(self._h, kappa, dt, theta, tau, nu1, nu2, tol, maxcyc, prec, coarse, solver,
                                 1 if unlimited else 0, _d(b), _d(x), C.byref(cyc))
        return rc, x, cyc.value

    def load_vector_fn(self, f) -> np.ndarray:
        """int f Phi_i dOmega for a Python function f(x, y) of the physical coordinates."""
        cb = FN2(f)
        out = np.zeros(self.ndof)
        lib().orc_load_vector_fn(self._h, cb, _d(out))
        return out

    def l2_error_fn(self, c: np.ndarray, u) -> float:
        c = np.ascontiguousarray(c, dtype=np.float64)
        return lib().orc_l2_error_fn(self._h, _d(c), FN2(u))

    def hmg_levels(self):
        ne = np.zeros(16, dtype=np.int32)
        nl = lib().orc_hmg_info(self._h, _i(ne))
        return [int(v) for v in ne[:nl]]

    def hmg_matrix(self, kappa, dt, k, which="A", theta=1.0):
        """h-multigrid level-k operator ("A") or prolongation P_k ("P") of A_{h,1}, scipy CSR."""
        import scipy.sparse as sp
        w = 0 if which == "A" else 1
        sh = np.zeros(3, dtype=np.int32)
        rc = lib().orc_hmg_matrix(self._h, kappa, dt, theta, k, w, _i(sh), None, None, None)
        if rc:
            raise ValueError(f"hmg_matrix failed: {rc}")
        nr, nc, nnz = (int(v) for v in sh)
        rp = np.zeros(nr + 1, dtype=np.int32)
        ci = np.zeros(max(nnz, 1), dtype=np.int32)
        v = np.zeros(max(nnz, 1))
        lib().orc_hmg_matrix(self._h, kappa, dt, theta, k, w, _i(sh), _i(rp), _i(ci), _d(v))
        return sp.csr_matrix((v[:nnz], ci[:nnz], rp), shape=(nr, nc))

    def hmg_cycles(self, kappa, dt, b, x0, ncyc, theta=1.0):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.array(x0, dtype=np.float64)
        rc = lib().orc_hmg_cycles(self._h, kappa, dt, theta, ncyc, _d(b), _d(x))
        if rc:
            raise RuntimeError(f"hmg failed: {rc}")
        return x

    def gs_sweep(self, kappa, dt, b, x0, direction=1, theta=1.0):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.array(x0, dtype=np.float64)
        lib().orc_gs_sweep(self._h, kappa, dt, theta, direction, _d(b), _d(x))
        return x

    def sequential(self, kappa: float, T: float, Nt: int, F: np.ndarray, tkind: int, u0: np.ndarray,
                   theta: float = 1.0):
        """Sequential theta-scheme with direct solves; returns U of shape (Nt+1, ndof)."""
        F = np.ascontiguousarray(F, dtype=np.float64)
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        U = np.zeros((Nt + 1, self.ndof))
        rc = lib().orc_sequential_theta(self._h, kappa, T, Nt, _d(F), tkind, theta, _d(u0), _d(U))
        if rc:
            raise RuntimeError(f"sequential solve failed: {rc}")
        return U

    def sequential_pmg(self, kappa, T, Nt, F, tkind, u0, tau=1e-12, stol=1e-12, maxcyc=100, theta=1.0, prec=0,
                       coarse=0, solver=0):
        F = np.ascontiguousarray(F, dtype=np.float64)
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        U = np.zeros((Nt + 1, self.ndof))
        cyc = C.c_longlong(0)
        rc = lib().orc_sequential_pmg(self._h, kappa, T, Nt, _d(F), tkind, theta, _d(u0), tau, stol, maxcyc, prec,
                                      coarse, solver, _d(U), C.byref(cyc))
        return rc, U, cyc.value

    def mgrit(self, kappa, T, Nt, F, tkind, u0, m=8, max_levels=30, coarsest_max=8, tol=1e-10,
              max_iter=100, tau=1e-12, stol=1e-12, maxcyc=100, guess=2, ctol=0.0, theta=1.0, cycle=0, prec=0,
              coarse=0, solver=0, threads=1):
        """MGRIT with the spatial solver above (level-0 tolerance stol, coarse levels ctol, 0 = stol);
        cycle 0 V, 1 W, 2 F; threads: OpenMP threads over the independent intervals of a sweep.
        Returns dict(rc, U, iters, cycles, solves, hist)."""
        F = np.ascontiguousarray(F, dtype=np.float64)
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        U = np.zeros((Nt + 1, self.ndof))
        it = C.c_int(0)
        cyc = C.c_longlong(0)
        sol = C.c_longlong(0)
        hist = np.zeros(200)
        iopt = np.array([m, max_levels, coarsest_max, max_iter, maxcyc, guess, cycle, prec, coarse, solver, threads],
                        dtype=np.int32)
        dopt = np.array([tol, tau, stol, ctol, theta], dtype=np.float64)
        rc = lib().orc_mgrit(self._h, kappa, T, Nt, _d(F), tkind, _d(u0), _i(iopt), _d(dopt), _d(U), C.byref(it),
                             C.byref(cyc), C.byref(sol), _d(hist))
        return dict(rc=rc, U=U, iters=it.value, cycles=cyc.value, solves=sol.value,
                    hist=hist[: it.value + 1].copy())
