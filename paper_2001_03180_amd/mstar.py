"""Thin ctypes binding of libmstar.so (include/mstar.h).

Argument marshalling only: every step of the integrator runs in the HIP
kernels of the library.  Arrays may be numpy float64 arrays (host memory) or
contiguous float64 torch CUDA tensors (device memory, passed with
MSTAR_DEVICE_PTRS).  The library must have been built
(paper_2001_03180_amd/build.py); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmstar.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_NONFINITE, E_COINCIDENT, E_NOCONV, E_MAXSTEPS, E_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
W_TIME_TOL = 1
DEVICE_PTRS = 1
EAGER = 2
MST_DC = 4          # divide-and-conquer spanning trees (Sec. 3.3) instead of the exact MST


class Params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("flags", C.c_uint32), ("G", C.c_double), ("eta", C.c_double),
        ("alpha", C.c_double), ("beta", C.c_double), ("gamma", C.c_double), ("omega_mass_max", C.c_double),
        ("a_gbs", C.c_double), ("f_min", C.c_double), ("f_max", C.c_double), ("q_first", C.c_double),
        ("t_tol", C.c_double), ("h_init", C.c_double), ("max_steps", C.c_int64), ("k_fix", C.c_int32),
        ("n_d", C.c_int32), ("max_halvings", C.c_int32), ("max_time_iter", C.c_int32),
        ("rebuild_every", C.c_int32), ("accept_rule", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("reserved", C.c_uint32), ("steps_accepted", C.c_int64),
        ("steps_rejected", C.c_int64), ("force_evals", C.c_int64), ("mst_rebuilds", C.c_int64),
        ("topo_changes", C.c_int64), ("time_iters", C.c_int64), ("t_reached", C.c_double),
        ("eps_last", C.c_double), ("h_next", C.c_double), ("h_last", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k not in ("struct_size", "reserved")}


class External(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_point", C.c_int32), ("g", C.c_double * 3),
                ("point", C.POINTER(C.c_double))]


MAX_EXT_POINTS = 16


class BatchConfig(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("wave_lanes", C.c_int32), ("wave_max_n", C.c_int32),
        ("wgs_per_cu", C.c_int32), ("use_graph", C.c_int32), ("reserved", C.c_int32), ("kernel_ms", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k not in ("struct_size", "reserved")}


# numpy mirror of mstar_batch_stats (one record per system)
BATCH_STATS_DTYPE = np.dtype([
    ("status", np.int32), ("reserved", np.int32), ("steps_accepted", np.int64), ("steps_rejected", np.int64),
    ("force_evals", np.int64), ("mst_rebuilds", np.int64), ("topo_changes", np.int64), ("time_iters", np.int64),
    ("t_reached", np.float64), ("eps_last", np.float64), ("h_next", np.float64), ("h_last", np.float64),
])

EXPORTS = {
    "mstar_abi_version": (C.c_int, []),
    "mstar_params_default": (None, [C.POINTER(Params)]),
    "mstar_strerror": (C.c_char_p, [C.c_int]),
    "mstar_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]),
    "mstar_destroy": (None, [C.c_void_p]),
    "mstar_last_error": (C.c_char_p, [C.c_void_p]),
    "mstar_integrate": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_double, C.c_double, C.POINTER(Stats)]),
    "mstar_integrate_ext": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_double, C.c_double, C.POINTER(External), C.POINTER(Stats)]),
    "mstar_mst_build": (C.c_int, [C.c_void_p, C.c_uint32, C.c_int64, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.c_void_p, C.c_void_p, C.c_void_p]),
    "mstar_force": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mstar_leapfrog": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_double, C.c_int32]),
    "mstar_gbs_step": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mstar_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "mstar_issue_rates": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mstar_rebuild_cycles": (C.c_int, [C.c_void_p, C.c_uint32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.POINTER(C.c_double)]),
    "mstar_profile_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]),
    "mstar_profile_read_kernel": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                            C.POINTER(C.c_double)]),
    "mstar_integrate_batch": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mstar_integrate_batch_record": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int32, C.c_void_p, C.c_void_p,
                                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                               C.c_int64, C.c_void_p]),
    "mstar_batch_get_config": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(BatchConfig)]),
    "mstar_batch_set_config": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(BatchConfig)]),
    "mstar_batch_autotune": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int32, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(BatchConfig)]),
    "mstar_integrate_record": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_double, C.c_double, C.c_int64, C.c_void_p,
                                         C.POINTER(C.c_int64), C.POINTER(Stats)]),
    "mstar_replay": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_double, C.c_int64, C.c_void_p, C.POINTER(C.c_double)]),
    "mstar_replay_adjoint": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_double, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p,
                                       C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mstar_integrate_adjoint": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_double, C.c_double, C.c_int64, C.c_int32, C.c_void_p,
                                          C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.POINTER(Stats)]),
    "mstar_adjoint_store_limit": (C.c_int, [C.c_void_p, C.c_int64]),
    "mstar_force_hvp": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "mstar_force_noalloc": (C.c_int, [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
}

_lib = None


def lib():
    """Load libmstar.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2001_03180_amd/build.py "
                               "(there is no CPU fallback)")
        _lib = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


class MstarError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mstar error {code}: {msg}")
        self.code = code


def params(**kw) -> Params:
    p = Params()
    lib().mstar_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _is_torch(a):
    return type(a).__module__.startswith("torch")


class _Arg:
    """Pointer to a float64 / int32 array, host (numpy) or device (torch)."""

    def __init__(self, a, dtype, shape=None, writable=False):
        self.obj = a
        if _is_torch(a):
            import torch
            want = torch.float64 if dtype == np.float64 else torch.int32
            if a.dtype != want or not a.is_contiguous() or not a.is_cuda:
                raise TypeError("device arrays must be contiguous CUDA tensors of the right dtype")
            if shape is not None and tuple(a.shape) != tuple(shape):
                raise ValueError(f"shape {tuple(a.shape)} != {shape}")
            self.dev = True
            self.ptr = C.c_void_p(a.data_ptr())
        else:
            if writable:
                if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags.c_contiguous):
                    raise TypeError("output arrays must be C-contiguous numpy arrays of the right dtype")
                arr = a
            else:
                arr = np.ascontiguousarray(a, dtype=dtype)
            if shape is not None and arr.shape != tuple(shape):
                raise ValueError(f"shape {arr.shape} != {shape}")
            self.arr = arr
            self.dev = False
            self.ptr = C.c_void_p(arr.ctypes.data)


def _mode(*args):
    devs = {a.dev for a in args}
    if len(devs) != 1:
        raise TypeError("mix of host and device arrays")
    if devs.pop():
        import torch
        torch.cuda.synchronize()
        return DEVICE_PTRS
    return 0


NOALLOC_MAX_N = 8192


def force_noalloc(m, rho, parent, X, acc, U, p: Params | None = None, stream=None):
    """mstar_force_noalloc on device tensors (m [n], rho [n,3], parent [n] int32,
    X [n,3] inputs; acc [n,3] and U [1] outputs, all on the current device):
    enqueues the evaluation on `stream` (a torch.cuda.Stream, default the
    current stream) without allocating; returns the status code."""
    import torch
    p = p or params()
    n = len(m)
    a = [_Arg(m, np.float64, (n,)), _Arg(rho, np.float64, (n, 3)), _Arg(parent, np.int32, (n,)),
         _Arg(X, np.float64, (n, 3)), _Arg(acc, np.float64, (n, 3), True), _Arg(U, np.float64, (1,), True)]
    if not all(x.dev for x in a):
        raise TypeError("force_noalloc takes device tensors only")
    s = (stream or torch.cuda.current_stream()).cuda_stream
    return lib().mstar_force_noalloc(C.c_void_p(s), C.byref(p), n, *(x.ptr for x in a))


class Context:
    """An mstar_ctx on one HIP device (own stream)."""

    def __init__(self, device: int = 0):
        self._h = C.c_void_p()
        rc = lib().mstar_create(C.byref(self._h), int(device), None)
        if rc != OK:
            raise MstarError(rc, lib().mstar_strerror(rc).decode())

    def close(self):
        if self._h:
            lib().mstar_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=(OK,)):
        if rc not in allow:
            raise MstarError(rc, lib().mstar_last_error(self._h).decode())
        return rc

    # ---------------------------------------------------------------- calls
    def mst_build(self, m, x, root_in=-1, dc=False):
        """MST of positions x rooted near the COM (dc: the divide-and-conquer
        tree of Sec. 3.3): (parent, level, root)."""
        n = len(m)
        M, X = _Arg(m, np.float64, (n,)), _Arg(x, np.float64, (n, 3))
        flags = _mode(M, X)
        if flags:
            import torch
            parent = torch.empty(n, dtype=torch.int32, device=x.device)
            level = torch.empty(n, dtype=torch.int32, device=x.device)
            root = torch.empty(1, dtype=torch.int32, device=x.device)
        else:
            parent, level, root = (np.empty(n, np.int32), np.empty(n, np.int32), np.empty(1, np.int32))
        P, L, R = (_Arg(parent, np.int32, writable=True), _Arg(level, np.int32, writable=True),
                   _Arg(root, np.int32, writable=True))
        self._check(lib().mstar_mst_build(self._h, flags | (MST_DC if dc else 0), n, M.ptr, X.ptr, int(root_in),
                                          P.ptr, L.ptr, R.ptr))
        return parent, level, int(root[0])

    def force(self, m, rho, parent, X, p: Params | None = None, omega: bool = False):
        """Accelerations [n,3] and force function U with MST separations; with
        omega=True also the TTL function Omega and its gradient [n,3] (zeros
        unless p.beta != 0): (acc, U, Omega, dOmega)."""
        p = p or params()
        n = len(m)
        args = [_Arg(m, np.float64, (n,)), _Arg(rho, np.float64, (n, 3)), _Arg(parent, np.int32, (n,)),
                _Arg(X, np.float64, (n, 3))]
        flags = _mode(*args)
        p.flags = flags
        if flags:
            import torch
            acc = torch.empty((n, 3), dtype=torch.float64, device=rho.device)
            U = torch.empty(2, dtype=torch.float64, device=rho.device)
            dOm = torch.empty((n, 3), dtype=torch.float64, device=rho.device) if omega else None
        else:
            acc, U = np.empty((n, 3)), np.empty(2)
            dOm = np.empty((n, 3)) if omega else None
        A, Ua = _Arg(acc, np.float64, writable=True), _Arg(U, np.float64, writable=True)
        Oa = _Arg(dOm, np.float64, writable=True) if omega else None
        om_ptr = C.c_void_p(Ua.ptr.value + 8) if omega else None   # U[1] receives Omega
        self._check(lib().mstar_force(self._h, C.byref(p), n, args[0].ptr, args[1].ptr, args[2].ptr,
                                      args[3].ptr, A.ptr, Ua.ptr, om_ptr, Oa.ptr if omega else None))
        if omega:
            return acc, float(U[0]), float(U[1]), dOm
        return acc, float(U[0])

    def leapfrog(self, m, parent, X, V, scal, H, nsub, p: Params | None = None):
        """One leapfrog division; returns new (X, V, scal) (host arrays are copied)."""
        p = p or params()
        n = len(m)
        X = np.array(X, dtype=np.float64) if not _is_torch(X) else X.clone()
        V = np.array(V, dtype=np.float64) if not _is_torch(V) else V.clone()
        scal = np.array(scal, dtype=np.float64) if not _is_torch(scal) else scal.clone()
        a = [_Arg(m, np.float64, (n,)), _Arg(parent, np.int32, (n,)), _Arg(X, np.float64, (n, 3), True),
             _Arg(V, np.float64, (n, 3), True), _Arg(scal, np.float64, (9,), True)]
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        self._check(lib().mstar_leapfrog(self._h, C.byref(p), n, a[0].ptr, a[1].ptr, a[2].ptr, a[3].ptr,
                                         a[4].ptr, float(H), int(nsub)))
        return X, V, scal

    def gbs_step(self, m, parent, X, V, scal, H, p: Params | None = None):
        """One GBS step: (X, V, scal, accepted, eps, h_next)."""
        p = p or params()
        n = len(m)
        X = np.array(X, dtype=np.float64) if not _is_torch(X) else X.clone()
        V = np.array(V, dtype=np.float64) if not _is_torch(V) else V.clone()
        scal = np.array(scal, dtype=np.float64) if not _is_torch(scal) else scal.clone()
        a = [_Arg(m, np.float64, (n,)), _Arg(parent, np.int32, (n,)), _Arg(X, np.float64, (n, 3), True),
             _Arg(V, np.float64, (n, 3), True), _Arg(scal, np.float64, (9,), True)]
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        acc, eps, hn = C.c_int32(), C.c_double(), C.c_double()
        self._check(lib().mstar_gbs_step(self._h, C.byref(p), n, a[0].ptr, a[1].ptr, a[2].ptr, a[3].ptr,
                                         a[4].ptr, float(H), C.cast(C.pointer(acc), C.c_void_p),
                                         C.cast(C.pointer(eps), C.c_void_p), C.cast(C.pointer(hn), C.c_void_p)))
        return X, V, scal, bool(acc.value), eps.value, hn.value

    def integrate(self, m, x, v, t0, t_end, p: Params | None = None, allow=(OK, W_TIME_TOL)):
        """Integrate in place-copy: returns (x, v, rc, stats dict)."""
        p = p or params()
        n = len(m)
        x = np.array(x, dtype=np.float64) if not _is_torch(x) else x.clone()
        v = np.array(v, dtype=np.float64) if not _is_torch(v) else v.clone()
        a = [_Arg(m, np.float64, (n,)), _Arg(x, np.float64, (n, 3), True), _Arg(v, np.float64, (n, 3), True)]
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        st = Stats()
        st.struct_size = C.sizeof(Stats)
        rc = lib().mstar_integrate(self._h, C.byref(p), n, a[0].ptr, a[1].ptr, a[2].ptr, float(t0), float(t_end),
                                   C.byref(st))
        self._check(rc, allow)
        return x, v, rc, st.as_dict()

    def integrate_ext(self, m, x, v, t0, t_end, g=(0.0, 0.0, 0.0), points=None, p: Params | None = None,
                      allow=(OK, W_TIME_TOL)):
        """integrate() under an external field: uniform acceleration g and
        fixed Plummer-softened point masses points[k] = (M, X, Y, Z, b)."""
        p = p or params()
        n = len(m)
        x = np.array(x, dtype=np.float64) if not _is_torch(x) else x.clone()
        v = np.array(v, dtype=np.float64) if not _is_torch(v) else v.clone()
        a = [_Arg(m, np.float64, (n,)), _Arg(x, np.float64, (n, 3), True), _Arg(v, np.float64, (n, 3), True)]
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        pts = np.ascontiguousarray(np.zeros((0, 5)) if points is None else np.asarray(points, dtype=np.float64)
                                   .reshape(-1, 5))
        e = External()
        e.struct_size = C.sizeof(External)
        e.n_point = len(pts)
        for c, gc in enumerate(np.asarray(g, dtype=np.float64).reshape(3)):
            e.g[c] = float(gc)
        e.point = pts.ctypes.data_as(C.POINTER(C.c_double)) if len(pts) else None
        st = Stats()
        st.struct_size = C.sizeof(Stats)
        rc = lib().mstar_integrate_ext(self._h, C.byref(p), n, a[0].ptr, a[1].ptr, a[2].ptr, float(t0), float(t_end),
                                       C.byref(e), C.byref(st))
        self._check(rc, allow)
        return x, v, rc, st.as_dict()

    # ---------------------------------------------------------------- batch
    def _batch_args(self, offsets, m, x, v, t_end, t0, copy):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        n_sys = len(off) - 1
        ntot = int(off[-1]) if n_sys >= 0 else 0
        te = np.ascontiguousarray(np.broadcast_to(np.asarray(t_end, dtype=np.float64), (n_sys,)))
        t0a = None if t0 is None else np.ascontiguousarray(np.broadcast_to(np.asarray(t0, dtype=np.float64),
                                                                            (n_sys,)))
        if copy:
            x = np.array(x, dtype=np.float64) if not _is_torch(x) else x.clone()
            v = np.array(v, dtype=np.float64) if not _is_torch(v) else v.clone()
        a = [_Arg(m, np.float64, (ntot,)), _Arg(x, np.float64, (ntot, 3), copy),
             _Arg(v, np.float64, (ntot, 3), copy)]
        return off, n_sys, te, t0a, x, v, a

    def integrate_batch(self, offsets, m, x, v, t_end, t0=None, p: Params | None = None):
        """Integrate n_sys independent systems (bodies offsets[s]..offsets[s+1]-1)
        to t_end[s] in one launch: returns (x, v, stats) with stats a numpy
        record array of BATCH_STATS_DTYPE (per-system status and counters)."""
        p = p or params()
        off, n_sys, te, t0a, x, v, a = self._batch_args(offsets, m, x, v, t_end, t0, True)
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        st = np.zeros(max(n_sys, 0), dtype=BATCH_STATS_DTYPE)
        self._check(lib().mstar_integrate_batch(
            self._h, C.byref(p), n_sys, C.c_void_p(off.ctypes.data), a[0].ptr, a[1].ptr, a[2].ptr,
            None if t0a is None else C.c_void_p(t0a.ctypes.data), C.c_void_p(te.ctypes.data),
            C.c_void_p(st.ctypes.data)))
        return x, v, st

    def integrate_batch_record(self, offsets, m, x, v, t_end, rec_cap, t0=None, p: Params | None = None):
        """integrate_batch that also records every system's accepted fictitious
        steps: (x, v, stats, H) with H[s, :stats['steps_accepted'][s]] valid."""
        p = p or params()
        off, n_sys, te, t0a, x, v, a = self._batch_args(offsets, m, x, v, t_end, t0, True)
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        st = np.zeros(max(n_sys, 0), dtype=BATCH_STATS_DTYPE)
        H = np.full((max(n_sys, 0), int(rec_cap)), np.nan)
        self._check(lib().mstar_integrate_batch_record(
            self._h, C.byref(p), n_sys, C.c_void_p(off.ctypes.data), a[0].ptr, a[1].ptr, a[2].ptr,
            None if t0a is None else C.c_void_p(t0a.ctypes.data), C.c_void_p(te.ctypes.data),
            C.c_void_p(st.ctypes.data), int(rec_cap), C.c_void_p(H.ctypes.data)))
        return x, v, st, H

    def batch_config(self, k_fix=8):
        c = BatchConfig()
        self._check(lib().mstar_batch_get_config(self._h, int(k_fix), C.byref(c)))
        return c.as_dict()

    def set_batch_config(self, k_fix=8, **kw):
        c = BatchConfig()
        self._check(lib().mstar_batch_get_config(self._h, int(k_fix), C.byref(c)))
        for k, val in kw.items():
            if not hasattr(c, k):
                raise KeyError(k)
            setattr(c, k, val)
        self._check(lib().mstar_batch_set_config(self._h, int(k_fix), C.byref(c)))
        return c.as_dict()

    def batch_autotune(self, offsets, m, x, v, t_end, t0=None, p: Params | None = None):
        """Time every launch shape on this batch (x, v untouched), keep and return the fastest."""
        p = p or params()
        off, n_sys, te, t0a, x, v, a = self._batch_args(offsets, m, x, v, t_end, t0, False)
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        c = BatchConfig()
        self._check(lib().mstar_batch_autotune(
            self._h, C.byref(p), n_sys, C.c_void_p(off.ctypes.data), a[0].ptr, a[1].ptr, a[2].ptr,
            None if t0a is None else C.c_void_p(t0a.ctypes.data), C.c_void_p(te.ctypes.data), C.byref(c)))
        return c.as_dict()

    # ---------------------------------------------------------------- replay / adjoint
    def integrate_record(self, m, x, v, t0, t_end, max_accepted, p: Params | None = None):
        """integrate() that records the fictitious step of every accepted step and
        stops after max_accepted of them: (x, v, rc, stats, H)."""
        p = p or params()
        n = len(m)
        x = np.array(x, dtype=np.float64) if not _is_torch(x) else x.clone()
        v = np.array(v, dtype=np.float64) if not _is_torch(v) else v.clone()
        a = [_Arg(m, np.float64, (n,)), _Arg(x, np.float64, (n, 3), True), _Arg(v, np.float64, (n, 3), True)]
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        H = np.zeros(int(max_accepted))
        k = C.c_int64()
        st = Stats()
        st.struct_size = C.sizeof(Stats)
        rc = lib().mstar_integrate_record(self._h, C.byref(p), n, a[0].ptr, a[1].ptr, a[2].ptr, float(t0),
                                          float(t_end), int(max_accepted), C.c_void_p(H.ctypes.data),
                                          C.byref(k), C.byref(st))
        self._check(rc, (OK, W_TIME_TOL))
        return x, v, rc, st.as_dict(), H[:k.value].copy()

    def replay(self, m, x, v, t0, H, p: Params | None = None):
        """Frozen-controller replay of the recorded steps H: (x, v, t)."""
        p = p or params()
        n = len(m)
        H = np.ascontiguousarray(H, dtype=np.float64)
        x = np.array(x, dtype=np.float64) if not _is_torch(x) else x.clone()
        v = np.array(v, dtype=np.float64) if not _is_torch(v) else v.clone()
        a = [_Arg(m, np.float64, (n,)), _Arg(x, np.float64, (n, 3), True), _Arg(v, np.float64, (n, 3), True)]
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        t = C.c_double()
        self._check(lib().mstar_replay(self._h, C.byref(p), n, a[0].ptr, a[1].ptr, a[2].ptr, float(t0), len(H),
                                       C.c_void_p(H.ctypes.data), C.byref(t)))
        return x, v, t.value

    def _grad_outputs(self, p, a, n, with_mass):
        if p.flags & DEVICE_PTRS:
            import torch
            dev = a[1].obj.device
            gx0 = torch.empty((n, 3), dtype=torch.float64, device=dev)
            gv0 = torch.empty((n, 3), dtype=torch.float64, device=dev)
            gm = torch.empty((n,), dtype=torch.float64, device=dev) if with_mass else None
        else:
            gx0, gv0 = np.empty((n, 3)), np.empty((n, 3))
            gm = np.empty(n) if with_mass else None
        o = [_Arg(gx0, np.float64, writable=True), _Arg(gv0, np.float64, writable=True)]
        om = _Arg(gm, np.float64, writable=True) if with_mass else None
        return gx0, gv0, gm, o, om

    def replay_adjoint(self, m, x0, v0, t0, H, gx, gv, gt=0.0, checkpoint_every=50, p: Params | None = None,
                       with_mass=False):
        """Gradient of <gx, x> + <gv, v> + gt t (end state of the replay) with
        respect to x0, v0: (gx0, gv0), and the masses (gm) with with_mass."""
        p = p or params()
        n = len(m)
        H = np.ascontiguousarray(H, dtype=np.float64)
        a = [_Arg(m, np.float64, (n,)), _Arg(x0, np.float64, (n, 3)), _Arg(v0, np.float64, (n, 3)),
             _Arg(gx, np.float64, (n, 3)), _Arg(gv, np.float64, (n, 3))]
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        gx0, gv0, gm, o, om = self._grad_outputs(p, a, n, with_mass)
        self._check(lib().mstar_replay_adjoint(self._h, C.byref(p), n, a[0].ptr, a[1].ptr, a[2].ptr, float(t0),
                                               len(H), C.c_void_p(H.ctypes.data), int(checkpoint_every),
                                               a[3].ptr, a[4].ptr, float(gt), o[0].ptr, o[1].ptr,
                                               om.ptr if om else None))
        return (gx0, gv0, gm) if with_mass else (gx0, gv0)

    def adjoint_store_limit(self, nbytes):
        """Bound (bytes) of the recomputed substep states the reverse pass keeps; 0 = default."""
        self._check(lib().mstar_adjoint_store_limit(self._h, int(nbytes)))

    def integrate_adjoint(self, m, x0, v0, t0, t_end, n_steps, gxT, gvT, gtT=0.0, checkpoint_every=50,
                          p: Params | None = None, with_mass=True):
        """Integrate n_steps accepted steps (or to t_end) and return the gradient
        of <gxT, x> + <gvT, v> + gtT t at the end with respect to x0, v0 and
        the masses: (gx0, gv0, gm, stats) (gm None without with_mass)."""
        p = p or params()
        n = len(m)
        a = [_Arg(m, np.float64, (n,)), _Arg(x0, np.float64, (n, 3)), _Arg(v0, np.float64, (n, 3)),
             _Arg(gxT, np.float64, (n, 3)), _Arg(gvT, np.float64, (n, 3))]
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        gx0, gv0, gm, o, om = self._grad_outputs(p, a, n, with_mass)
        st = Stats()
        st.struct_size = C.sizeof(Stats)
        rc = lib().mstar_integrate_adjoint(self._h, C.byref(p), n, a[0].ptr, a[1].ptr, a[2].ptr, float(t0),
                                           float(t_end), int(n_steps), int(checkpoint_every), a[3].ptr, a[4].ptr,
                                           float(gtT), o[0].ptr, o[1].ptr, om.ptr if om else None, C.byref(st))
        self._check(rc, (OK, W_TIME_TOL))
        return gx0, gv0, gm, st.as_dict()

    def force_hvp(self, m, x, w, p: Params | None = None):
        """out_i = G sum_j M(d_ij)(m_i w_j - m_j w_i): the transposed Jacobian of the accelerations times w."""
        p = p or params()
        n = len(m)
        a = [_Arg(m, np.float64, (n,)), _Arg(x, np.float64, (n, 3)), _Arg(w, np.float64, (n, 3))]
        p.flags = (p.flags & ~DEVICE_PTRS) | _mode(*a)
        if p.flags:
            import torch
            out = torch.empty((n, 3), dtype=torch.float64, device=a[1].obj.device)
        else:
            out = np.empty((n, 3))
        o = _Arg(out, np.float64, writable=True)
        self._check(lib().mstar_force_hvp(self._h, C.byref(p), n, a[0].ptr, a[1].ptr, a[2].ptr, o.ptr))
        return out

    def rebuild_cycles(self, offsets, kinds, m, x, v, n_cycles, n_out):
        """Coordinate round trips (kind 0 MST, 1 chain per system): returns the
        states after cycles (k+1) n_cycles / n_out as [n_out, n_tot, 3] arrays
        and each system's mean structure level over the cycles."""
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        n_sys = len(off) - 1
        kd = np.ascontiguousarray(kinds, dtype=np.int32)
        n_tot = int(off[-1])
        a = [_Arg(m, np.float64, (n_tot,)), _Arg(x, np.float64, (n_tot, 3)), _Arg(v, np.float64, (n_tot, 3))]
        flags = _mode(*a)
        if flags:
            import torch
            dev = a[1].obj.device
            xo = torch.empty((max(n_out, 1), n_tot, 3), dtype=torch.float64, device=dev)
            vo = torch.empty((max(n_out, 1), n_tot, 3), dtype=torch.float64, device=dev)
            doff = torch.tensor(off, device=dev)
            dkd = torch.tensor(kd, device=dev)
            po, pk = C.c_void_p(doff.data_ptr()), C.c_void_p(dkd.data_ptr())
        else:
            xo = np.empty((max(n_out, 1), n_tot, 3))
            vo = np.empty((max(n_out, 1), n_tot, 3))
            po, pk = C.c_void_p(off.ctypes.data), C.c_void_p(kd.ctypes.data)
        X, V = _Arg(xo, np.float64, writable=True), _Arg(vo, np.float64, writable=True)
        ml = np.empty(n_sys)
        self._check(lib().mstar_rebuild_cycles(self._h, flags, n_sys, po, pk, a[0].ptr, a[1].ptr, a[2].ptr,
                                               int(n_cycles), int(n_out), X.ptr, V.ptr,
                                               ml.ctypes.data_as(C.POINTER(C.c_double))))
        return xo[:n_out], vo[:n_out], ml

    def issue_rates(self):
        """(SIMD cycles per wave-level FP64 FMA, per hardware 1/sqrt) at the nominal 2.4 GHz."""
        f, r = C.c_double(), C.c_double()
        self._check(lib().mstar_issue_rates(self._h, C.byref(f), C.byref(r)))
        return f.value, r.value

    def profile_enable(self, on=True):
        self._check(lib().mstar_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """(force launches, summed force-kernel ms, directed pairs) since enable."""
        L, ms, pairs = C.c_int64(), C.c_double(), C.c_double()
        self._check(lib().mstar_profile_read(self._h, C.byref(L), C.byref(ms), C.byref(pairs)))
        return L.value, ms.value, pairs.value

    def profile_read_kernel(self, kind):
        """The same for one force kernel: kind 0 pairwise, 1 mutual."""
        L, ms, pairs = C.c_int64(), C.c_double(), C.c_double()
        self._check(lib().mstar_profile_read_kernel(self._h, int(kind), C.byref(L), C.byref(ms), C.byref(pairs)))
        return L.value, ms.value, pairs.value
