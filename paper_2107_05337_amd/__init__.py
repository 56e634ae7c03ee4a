"""Python binding of libpmgrit.so (include/pmgrit.h): argument marshalling only.

Every step of the solver runs in the library's HIP kernels; PyTorch supplies device memory
(tensor data pointers) and streams.  Importing this package does not need a GPU; calling a
solve does, and fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmgrit.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pmgrit.h")

STATUS = {0: "OK", -1: "E_ARG", -2: "E_HIP", -3: "E_OOM", -4: "E_FACTOR", -5: "E_SPATIAL_NOCONV",
          -6: "E_MGRIT_NOCONV", -7: "E_NONFINITE", -8: "E_STATE"}


class PmgritError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pmgrit {STATUS.get(code, code)}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [("degree_p", C.c_int32), ("n_elems", C.c_int32), ("domain", C.c_int32), ("kappa", C.c_double),
                ("T", C.c_double), ("n_steps", C.c_int32), ("theta", C.c_double)]


class MgritOpts(C.Structure):
    _fields_ = [("cfactor", C.c_int32), ("max_levels", C.c_int32), ("coarsest_max", C.c_int32),
                ("tol", C.c_double), ("max_iter", C.c_int32), ("use_graph", C.c_int32), ("cycle", C.c_int32)]


class SolverOpts(C.Structure):
    _fields_ = [("nu1", C.c_int32), ("nu2", C.c_int32), ("ilut_droptol", C.c_double), ("ilut_fill", C.c_int32),
                ("spatial_tol", C.c_double), ("max_vcycles", C.c_int32), ("precision", C.c_int32),
                ("guess", C.c_int32), ("trsv_block", C.c_int32), ("autotune", C.c_int32),
                ("coarse_tol", C.c_double), ("lds_mask", C.c_int32), ("solver", C.c_int32),
                ("coarse", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("mgrit_iters", C.c_int32), ("res_hist", C.c_double * 64), ("phi_calls", C.c_int64),
                ("vcycles", C.c_int64), ("t_setup_s", C.c_double), ("t_solve_s", C.c_double)]

    def as_dict(self):
        it = self.mgrit_iters
        return dict(mgrit_iters=it, res_hist=list(self.res_hist[: min(it + 1, 64)]), phi_calls=self.phi_calls,
                    vcycles=self.vcycles, t_setup_s=self.t_setup_s, t_solve_s=self.t_solve_s)


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("seed", C.c_uint32)]


class TrainStats(C.Structure):
    _fields_ = [("epochs_done", C.c_int32), ("adam_steps", C.c_int64), ("loss_first", C.c_double),
                ("loss_last", C.c_double), ("seconds", C.c_double)]


_lib = None
_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_fp = C.POINTER(C.c_float)


def lib():
    """Load libpmgrit.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() or paper_2107_05337_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.pmgrit_create.argtypes = [C.c_int32, C.POINTER(Problem), C.POINTER(MgritOpts), C.POINTER(SolverOpts),
                                    C.c_int32, C.POINTER(_vp)]
        L.pmgrit_create.restype = C.c_int
        L.pmgrit_destroy.argtypes = [_vp]
        L.pmgrit_destroy.restype = None
        L.pmgrit_dims.argtypes = [_vp, C.c_int32, C.POINTER(C.c_int64), _ip, _ip]
        L.pmgrit_set_source_modes.argtypes = [_vp, C.c_int32, C.c_int32, _ip, _ip, _dp, C.c_int32]
        L.pmgrit_set_initial_modes.argtypes = [_vp, C.c_int32, C.c_int32, _ip, _ip, _dp]
        L.pmgrit_set_initial_coeffs.argtypes = [_vp, C.c_int32, _dp]
        L.pmgrit_solve_mgrit.argtypes = [_vp, _vp, C.POINTER(_vp), C.POINTER(Stats)]
        L.pmgrit_solve_sequential.argtypes = [_vp, _vp, C.POINTER(_vp), C.POINTER(Stats)]
        L.pmgrit_phi.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp]
        L.pmgrit_phi_noalloc.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp]
        L.pmgrit_host_matrix.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int32, _ip, _ip, _ip, _dp]
        L.pmgrit_host_vectors.argtypes = [_vp, C.c_int32, _dp, _dp, _dp, _dp]
        L.pmgrit_host_schedule.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int32, _ip]
        L.pmgrit_host_coarse_solve.argtypes = [_vp, C.c_int32, C.c_int32, _dp, _dp]
        L.pmgrit_info.argtypes = [_vp, C.POINTER(C.c_int64)]
        L.pmgrit_group_info.argtypes = [_vp, C.c_int32, C.POINTER(C.c_int64)]
        L.pmgrit_profile.argtypes = [_vp, C.c_int32, _dp]
        L.pmgrit_group_profile.argtypes = [_vp, C.c_int32, _dp]
        L.pmgrit_inst_vcycles.argtypes = [_vp, C.POINTER(C.c_int64)]
        L.pmgrit_net_nparams.argtypes = []
        L.pmgrit_net_nparams.restype = C.c_int64
        L.pmgrit_net_load.argtypes = [_vp, _fp, C.c_int64]
        L.pmgrit_net_save.argtypes = [_vp, _fp, C.c_int64]
        L.pmgrit_net_forward.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp]
        L.pmgrit_net_grad.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, _fp, _dp, _vp]
        L.pmgrit_net_train_step.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, C.c_float, _dp, _vp]
        L.pmgrit_net_pack.argtypes = [_vp, C.c_int32, C.c_int32, C.c_int32, _ip, _vp, _vp, _vp, _vp, _vp]
        L.pmgrit_net_train.argtypes = [_vp, C.POINTER(TrainOpts), C.POINTER(_vp), _vp, C.POINTER(TrainStats)]
        L.pmgrit_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise PmgritError(rc, lib().pmgrit_last_error().decode())


def header_functions() -> list[str]:
    """Names of the functions include/pmgrit.h declares."""
    import re
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:pmgrit_status|void|int64_t|const char\*)\s+(pmgrit_\w+)\s*\(", txt, re.M)))


def _stream_ptr(stream, device: int = 0):
    if stream is None and device < 0:
        return 0
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _dptr(t):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA/HIP torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def default_solver_opts(**kw) -> SolverOpts:
    o = SolverOpts(nu1=1, nu2=1, ilut_droptol=1e-12, ilut_fill=0, spatial_tol=1e-12, max_vcycles=100, precision=0,
                   guess=2, trsv_block=0, autotune=0, coarse_tol=0.0, lds_mask=0, solver=0, coarse=0)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_mgrit_opts(**kw) -> MgritOpts:
    o = MgritOpts(cfactor=8, max_levels=12, coarsest_max=8, tol=1e-10, max_iter=100, use_graph=0, cycle=0)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Solver:
    """One handle: n instances sharing N_t and the MGRIT / solver options."""

    def __init__(self, problems, mgrit: MgritOpts | None = None, solver: SolverOpts | None = None, device: int = 0):
        arr = (Problem * len(problems))(*problems)
        self.mgrit = mgrit or default_mgrit_opts()
        self.solver = solver or default_solver_opts()
        h = _vp()
        _check(lib().pmgrit_create(len(problems), arr, C.byref(self.mgrit), C.byref(self.solver), device, C.byref(h)))
        self._h = h
        self.n = len(problems)
        self.problems = list(problems)
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().pmgrit_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dims(self, inst: int = 0):
        nd = C.c_int64()
        g = C.c_int32()
        nl = C.c_int32()
        _check(lib().pmgrit_dims(self._h, inst, C.byref(nd), C.byref(g), C.byref(nl)))
        return nd.value, g.value, nl.value

    def info(self):
        out = (C.c_int64 * 8)()
        _check(lib().pmgrit_info(self._h, out))
        keys = ["precision", "lds_mask", "lds_bytes", "device_lds", "ws_stride", "slots", "levels", "instances"]
        return dict(zip(keys, list(out)))

    def group_info(self, inst: int = 0):
        """Launch group of instance inst: dict(group, groups, lds_mask, lds_mask_wide, lds_bytes, ka,
        size, nmax, slots); lds_mask_wide is the placement of sweeps wider than the device's CUs."""
        out = (C.c_int64 * 8)()
        _check(lib().pmgrit_group_info(self._h, inst, out))
        keys = ["group", "groups", "lds_mask", "lds_bytes", "ka", "size", "nmax", "slots"]
        d = dict(zip(keys, list(out)))
        d["lds_mask_wide"] = d["lds_mask"] >> 8
        d["lds_mask"] &= 0xFF
        return d

    def profile(self, enable: int = -1):
        """Live kernel timing: enable 1 resets and starts, 0 stops, -1 only reads.  Returns
        dict(ms, launches, workgroups, vcycles) accumulated since the last reset."""
        out = (C.c_double * 4)()
        _check(lib().pmgrit_profile(self._h, enable, out))
        return dict(ms=out[0], launches=int(out[1]), workgroups=int(out[2]), vcycles=int(out[3]))

    def group_profile(self, group: int):
        """Per-launch timing of one launch group since the last profile reset: dict(ms, launches,
        workgroups)."""
        out = (C.c_double * 3)()
        _check(lib().pmgrit_group_profile(self._h, group, out))
        return dict(ms=out[0], launches=int(out[1]), workgroups=int(out[2]))

    def inst_vcycles(self):
        """V-cycles (or CG iterations) per instance since create."""
        out = (C.c_int64 * self.n)()
        _check(lib().pmgrit_inst_vcycles(self._h, out))
        return [int(v) for v in out]

    @staticmethod
    def _modes(modes):
        k = np.ascontiguousarray([m[0] for m in modes], dtype=np.int32)
        l_ = np.ascontiguousarray([m[1] for m in modes], dtype=np.int32)
        a = np.ascontiguousarray([m[2] for m in modes], dtype=np.float64)
        return k, l_, a

    def set_source(self, inst: int, modes, time_kind: int = 0):
        k, l_, a = self._modes(modes)
        _check(lib().pmgrit_set_source_modes(self._h, inst, len(modes), k.ctypes.data_as(_ip), l_.ctypes.data_as(_ip),
                                             a.ctypes.data_as(_dp), time_kind))

    def set_initial_modes(self, inst: int, modes):
        k, l_, a = self._modes(modes)
        _check(lib().pmgrit_set_initial_modes(self._h, inst, len(modes), k.ctypes.data_as(_ip),
                                              l_.ctypes.data_as(_ip), a.ctypes.data_as(_dp)))

    def set_initial_coeffs(self, inst: int, u0):
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        _check(lib().pmgrit_set_initial_coeffs(self._h, inst, u0.ctypes.data_as(_dp)))

    def _outs(self, outs):
        if self.device < 0:
            return (_vp * self.n)()
        if len(outs) != self.n:
            raise ValueError("one trajectory buffer per instance")
        ptrs = (_vp * self.n)(*[_dptr(t) for t in outs])
        return ptrs

    def alloc_trajectories(self):
        import torch
        out = []
        for i in range(self.n):
            nd, _, _ = self.dims(i)
            out.append(torch.zeros((self.problems[i].n_steps + 1, nd), dtype=torch.float64,
                                   device=f"cuda:{self.device}"))
        return out

    def solve_mgrit(self, outs=None, stream=None):
        outs = outs if outs is not None or self.device < 0 else self.alloc_trajectories()
        st = Stats()
        _check(lib().pmgrit_solve_mgrit(self._h, _vp(_stream_ptr(stream, self.device)), self._outs(outs),
                                        C.byref(st)))
        return outs, st.as_dict()

    def solve_sequential(self, outs=None, stream=None):
        outs = outs if outs is not None else self.alloc_trajectories()
        st = Stats()
        _check(lib().pmgrit_solve_sequential(self._h, _vp(_stream_ptr(stream, self.device)), self._outs(outs),
                                             C.byref(st)))
        return outs, st.as_dict()

    def phi(self, inst: int, level: int, b, x, vcycles=None, stream=None):
        nrhs = b.shape[0]
        vc = _dptr(vcycles) if vcycles is not None else _vp()
        _check(lib().pmgrit_phi(self._h, inst, level, nrhs, _dptr(b), _dptr(x), vc, _vp(_stream_ptr(stream))))
        return x

    def phi_noalloc(self, inst: int, level: int, b, x, vcycles=None, stream=None):
        """pmgrit_phi with the kernels' scratch in the library's fixed device array (no allocation)"""
        nrhs = b.shape[0]
        vc = _dptr(vcycles) if vcycles is not None else _vp()
        _check(lib().pmgrit_phi_noalloc(self._h, inst, level, nrhs, _dptr(b), _dptr(x), vc,
                                        _vp(_stream_ptr(stream))))
        return x

    # ---- learned warm start ----
    @staticmethod
    def net_nparams() -> int:
        return int(lib().pmgrit_net_nparams())

    def net_load(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        _check(lib().pmgrit_net_load(self._h, th.ctypes.data_as(_fp), th.size))

    def net_save(self):
        th = np.zeros(self.net_nparams(), dtype=np.float32)
        _check(lib().pmgrit_net_save(self._h, th.ctypes.data_as(_fp), th.size))
        return th

    def net_forward(self, x, y=None, stream=None):
        """x: (nb, 3, G, G) float32 CUDA tensor -> y (nb, G, G)."""
        import torch
        nb, _, G, _ = x.shape
        y = y if y is not None else torch.empty((nb, G, G), dtype=torch.float32, device=x.device)
        _check(lib().pmgrit_net_forward(self._h, G, nb, _dptr(x), _dptr(y), _vp(_stream_ptr(stream))))
        return y

    def net_grad(self, x, t, stream=None):
        nb, _, G, _ = x.shape
        g = np.zeros(self.net_nparams(), dtype=np.float32)
        loss = C.c_double()
        _check(lib().pmgrit_net_grad(self._h, G, nb, _dptr(x), _dptr(t), g.ctypes.data_as(_fp), C.byref(loss),
                                     _vp(_stream_ptr(stream))))
        return loss.value, g

    def net_train_step(self, x, t, lr: float, stream=None):
        nb, _, G, _ = x.shape
        loss = C.c_double()
        _check(lib().pmgrit_net_train_step(self._h, G, nb, _dptr(x), _dptr(t), lr, C.byref(loss),
                                           _vp(_stream_ptr(stream))))
        return loss.value

    def net_pack(self, inst: int, level: int, ks, U, with_target: bool = True, stream=None):
        """Planes (nb, 3, G, G), targets (nb, G, G) or None, scales (nb,) of samples (inst, k -> k+1)."""
        import torch
        ks = np.ascontiguousarray(ks, dtype=np.int32)
        nb = ks.size
        p = self.problems[inst]
        G = p.n_elems + p.degree_p
        dev = U.device
        x = torch.empty((nb, 3, G, G), dtype=torch.float32, device=dev)
        t = torch.empty((nb, G, G), dtype=torch.float32, device=dev) if with_target else None
        s = torch.empty(nb, dtype=torch.float64, device=dev)
        _check(lib().pmgrit_net_pack(self._h, inst, level, nb, ks.ctypes.data_as(_ip), _dptr(U), _dptr(x),
                                     _dptr(t) if t is not None else _vp(), _dptr(s), _vp(_stream_ptr(stream))))
        return x, t, s

    def net_train(self, trajectories, epochs: int, batch: int, lr: float, seed: int = 0, stream=None):
        o = TrainOpts(epochs=epochs, batch=batch, lr=lr, seed=seed)
        st = TrainStats()
        ptrs = (_vp * self.n)(*[_dptr(u) for u in trajectories])
        _check(lib().pmgrit_net_train(self._h, C.byref(o), ptrs, _vp(_stream_ptr(stream)), C.byref(st)))
        return dict(epochs=st.epochs_done, adam_steps=st.adam_steps, loss_first=st.loss_first,
                    loss_last=st.loss_last, seconds=st.seconds)

    # ---- host inspection ----
    MATS = {"M": 0, "K": 1, "A": 2, "L": 3, "U": 4, "P": 5, "M1": 6, "K1": 7}

    def host_matrix(self, name: str, inst: int = 0, level: int = 0):
        import scipy.sparse as sp
        sh = (C.c_int32 * 3)()
        w = self.MATS[name]
        _check(lib().pmgrit_host_matrix(self._h, inst, level, w, sh, None, None, None))
        nr, nc, nnz = sh
        rp = np.zeros(nr + 1, dtype=np.int32)
        ci = np.zeros(max(nnz, 1), dtype=np.int32)
        v = np.zeros(max(nnz, 1))
        _check(lib().pmgrit_host_matrix(self._h, inst, level, w, sh, rp.ctypes.data_as(_ip), ci.ctypes.data_as(_ip),
                                        v.ctypes.data_as(_dp)))
        return sp.csr_matrix((v[:nnz], ci[:nnz], rp), shape=(nr, nc))

    def host_vectors(self, inst: int = 0):
        nd, g, _ = self.dims(inst)
        p = self.problems[inst]
        nd1 = (p.n_elems - 1) ** 2
        mlp, ml1, load, u0 = np.zeros(nd), np.zeros(nd1), np.zeros(nd), np.zeros(nd)
        _check(lib().pmgrit_host_vectors(self._h, inst, mlp.ctypes.data_as(_dp), ml1.ctypes.data_as(_dp),
                                         load.ctypes.data_as(_dp), u0.ctypes.data_as(_dp)))
        return dict(mlp=mlp, ml1=ml1, load=load, u0=u0)

    def host_schedule(self, inst: int = 0, level: int = 0, factor: int = 0):
        out = (C.c_int32 * 4)()
        _check(lib().pmgrit_host_schedule(self._h, inst, level, factor, out))
        return dict(levels=out[0], blocks=out[1], block_size=out[2], max_rows=out[3])

    def host_coarse_solve(self, b, inst: int = 0, level: int = 0):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        _check(lib().pmgrit_host_coarse_solve(self._h, inst, level, b.ctypes.data_as(_dp), x.ctypes.data_as(_dp)))
        return x


def problem(p: int, n: int, Nt: int, kappa: float = 1.0, T: float = 0.1, domain: int = 0,
            theta: float = 1.0) -> Problem:
    return Problem(degree_p=p, n_elems=n, domain=domain, kappa=kappa, T=T, n_steps=Nt, theta=theta)
