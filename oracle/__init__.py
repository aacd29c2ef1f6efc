"""CPU FP64 oracle of the MSTAR integrator -- TEST INFRASTRUCTURE.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this package.  It wraps the plain C implementation in mstar_oracle.c
(built into liborc.so by oracle/build.py) with numpy marshalling, and adds
pure-Python reference routines used as independent pins.  It shares no code
with the GPU library and never imports it.

State convention (MST coordinates, paper Sec. 2.2 and 3.4): parent[n] (int32,
root = -1), X[n,3] and V[n,3] (row v = edge vector from parent(v) to v, root
row zero), scal[9] = (t, B, w, r_cm[3], v_cm[3]).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MSTAR_ORACLE_LIB selects another build of the same source (the sanitizer test)
_LIB = os.environ.get("MSTAR_ORACLE_LIB") or os.path.join(_HERE, "liborc.so")

OK, E_INVAL, E_NOMEM, E_NONFINITE, E_COINCIDENT, E_NOCONV, E_MAXSTEPS = 0, -1, -2, -4, -5, -6, -7
W_TIME_TOL = 1


class Params(C.Structure):
    _fields_ = [
        ("G", C.c_double), ("eta", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
        ("gamma", C.c_double), ("omega_mass_max", C.c_double), ("a_gbs", C.c_double),
        ("f_min", C.c_double), ("f_max", C.c_double), ("q_first", C.c_double), ("t_tol", C.c_double),
        ("h_init", C.c_double), ("max_steps", C.c_int64), ("k_fix", C.c_int32), ("n_d", C.c_int32),
        ("max_halvings", C.c_int32), ("max_time_iter", C.c_int32), ("rebuild_every", C.c_int32),
        ("nthreads", C.c_int32), ("accept_rule", C.c_int32), ("mst_method", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("steps_accepted", C.c_int64), ("steps_rejected", C.c_int64), ("force_evals", C.c_int64),
        ("mst_rebuilds", C.c_int64), ("topo_changes", C.c_int64), ("time_iters", C.c_int64),
        ("t_reached", C.c_double), ("eps_last", C.c_double), ("h_next", C.c_double), ("h_last", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def params(**kw) -> Params:
    """Default parameters (LogH, k_fix = 8, N_d = 2, eta = 1e-12), overridable."""
    p = Params(G=1.0, eta=1e-12, alpha=1.0, beta=0.0, gamma=0.0, omega_mass_max=0.0, a_gbs=0.9,
               f_min=0.1, f_max=4.0, q_first=0.1, t_tol=1e-14, h_init=0.0, max_steps=10**9, k_fix=8,
               n_d=2, max_halvings=60, max_time_iter=8, rebuild_every=1, nthreads=0, accept_rule=0,
               mst_method=0)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(_LIB)
        D, I, I64 = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        P = C.POINTER(Params)
        sig = {
            "orc_root_nearest_com": (C.c_int, [C.c_int, D, D]),
            "orc_mst_prim": (C.c_int, [C.c_int, D, C.c_int, I, I, I]),
            "orc_mst_dc": (C.c_int, [C.c_int, D, C.c_int, C.c_int, I, I, I, I, I]),
            "orc_chain_build": (C.c_int, [C.c_int, D, I, I, I]),
            "orc_rebuild_cycles": (C.c_int, [C.c_int, D, D, D, C.c_int, C.c_int64, C.c_int, D, D, D]),
            "orc_tree_levels": (C.c_int, [C.c_int, I, I, I]),
            "orc_deconstruct": (None, [C.c_int, I, I, D, D]),
            "orc_separation": (C.c_int, [C.c_int, C.c_int, I, I, D, D, C.c_int, D]),
            "orc_force_tree": (C.c_int, [C.c_int, D, I, D, D, P, D, D, D, D, D]),
            "orc_leapfrog": (C.c_int, [C.c_int, D, I, D, D, D, P, C.c_double, C.c_int, I64]),
            "orc_gbs_step": (C.c_int, [C.c_int, D, I, D, D, D, P, C.c_double, I, D, D, I64]),
            "orc_neville_export": (C.c_int, [C.c_int, C.c_int, D, D]),
            "orc_build_state": (C.c_int, [C.c_int, D, D, D, I, D, D, D]),
            "orc_state_to_cartesian": (C.c_int, [C.c_int, D, I, D, D, D, D, D]),
            "orc_integrate": (C.c_int, [C.c_int, D, D, D, C.c_double, C.c_double, P, C.POINTER(Stats)]),
            "orc_integrate_ext": (C.c_int, [C.c_int, D, D, D, C.c_double, C.c_double, P, C.c_int, D, D,
                                            C.POINTER(Stats)]),
            "orc_external_accel": (C.c_int, [C.c_int, D, D, C.c_double, C.c_int, D, D]),
            "orc_diagnostics": (None, [C.c_int, D, D, D, C.c_double, D]),
            "orc_sdiv": (C.c_double, [C.c_int, C.c_int, I]),
            "orc_integrate_rec": (C.c_int, [C.c_int, D, D, D, C.c_double, C.c_double, P, C.POINTER(Stats),
                                            C.c_int64, D, I, I64]),
            "orc_replay": (C.c_int, [C.c_int, D, D, D, C.c_double, C.c_int64, D, I, P, D, D]),
            "orc_rebuild_state": (C.c_int, [C.c_int, D, I, D, D, D, P, I]),
            "orc_force_tlm": (C.c_int, [C.c_int, D, D, C.c_double, C.c_int, D, D, D, D, D, C.c_int]),
            "orc_lagrange_weights": (None, [C.c_int, D]),
            "orc_replay_tlm": (C.c_int, [C.c_int, D, D, D, C.c_double, C.c_int64, D, P, C.c_int, D, D, D, D]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


# ---------------------------------------------------------------- stages
def root_nearest_com(m, x) -> int:
    m, pm = _d(m)
    x, px = _d(x)
    return lib().orc_root_nearest_com(len(m), pm, px)


def mst(x, root):
    """Prim MST rooted at `root`: returns (parent, level, order)."""
    x, px = _d(x)
    n = x.shape[0]
    parent, pp = _i(np.empty(n, dtype=np.int32))
    level, pl = _i(np.empty(n, dtype=np.int32))
    order, po = _i(np.empty(n, dtype=np.int32))
    _check(lib().orc_mst_prim(n, px, int(root), pp, pl, po), "mst")
    return parent, level, order


def mst_dc(x, root, mcap=0):
    """Divide-and-conquer spanning tree (Sec. 3.3) rooted at `root`, groups of at
    most mcap bodies (0: ceil(sqrt(N))): returns (parent, level, order, part, nparts)."""
    x, px = _d(x)
    n = x.shape[0]
    parent, pp = _i(np.empty(n, dtype=np.int32))
    level, pl = _i(np.empty(n, dtype=np.int32))
    order, po = _i(np.empty(n, dtype=np.int32))
    part, pq = _i(np.empty(n, dtype=np.int32))
    npart = np.zeros(1, dtype=np.int32)
    _check(lib().orc_mst_dc(n, px, int(root), int(mcap), pp, pl, po, pq,
                            npart.ctypes.data_as(C.POINTER(C.c_int32))), "mst_dc")
    return parent, level, order, part, int(npart[0])


def chain(x):
    """Greedy chain of Sec. 2.2 as a tree rooted at its tail: (parent, level, order)."""
    x, px = _d(x)
    n = len(x)
    parent, pp = _i(np.empty(n, dtype=np.int32))
    level, pl = _i(np.empty(n, dtype=np.int32))
    order, po = _i(np.empty(n, dtype=np.int32))
    _check(lib().orc_chain_build(n, px, pp, pl, po), "chain")
    return parent, level, order


def rebuild_cycles(m, x, v, kind, n_cycles, n_out):
    """Sec. 3.5 rebuild test: n_cycles build / deconstruct round trips (kind 0
    MST, 1 chain; + 2: plain centre-of-mass sums in index order instead of
    compensated ones).  Returns the states after cycles (k+1) n_cycles / n_out,
    shape [n_out, n, 3] each, and the mean level of the structure averaged
    over the cycles."""
    m, pm = _d(m)
    x = np.array(x, dtype=np.float64, order="C")
    v = np.array(v, dtype=np.float64, order="C")
    n = len(m)
    xs = np.empty((max(n_out, 1), n, 3))
    vs = np.empty((max(n_out, 1), n, 3))
    ls = C.c_double()
    _check(lib().orc_rebuild_cycles(n, pm, _d(x)[1], _d(v)[1], int(kind), int(n_cycles), int(n_out),
                                    _d(xs)[1], _d(vs)[1], C.byref(ls)), "rebuild_cycles")
    return xs[:n_out], vs[:n_out], ls.value / max(n_cycles, 1)


def tree_levels(parent):
    parent, pp = _i(parent)
    n = parent.shape[0]
    level, pl = _i(np.empty(n, dtype=np.int32))
    order, po = _i(np.empty(n, dtype=np.int32))
    root = lib().orc_tree_levels(n, pp, pl, po)
    if root < 0:
        raise ValueError("not a rooted tree")
    return root, level, order


def deconstruct(parent, X):
    _, level, order = tree_levels(parent)
    parent, pp = _i(parent)
    X, pX = _d(X)
    rho = np.empty_like(X)
    _, prho = _d(rho)
    lib().orc_deconstruct(len(parent), pp, order.ctypes.data_as(C.POINTER(C.c_int32)), pX, prho)
    return rho


def separation(i, j, parent, X, rho, n_d=2):
    _, level, _ = tree_levels(parent)
    parent, pp = _i(parent)
    X, pX = _d(X)
    rho, pr = _d(rho)
    d = np.empty(3)
    _, pd = _d(d)
    close = lib().orc_separation(int(i), int(j), pp, level.ctypes.data_as(C.POINTER(C.c_int32)), pX, pr,
                                 int(n_d), pd)
    return d, bool(close)


def force(m, parent, X, rho, p: Params | None = None):
    """Accelerations, phi, U, Omega, dOmega with MST separations."""
    p = p or params()
    m, pm = _d(m)
    parent, pp = _i(parent)
    X, pX = _d(X)
    rho, pr = _d(rho)
    n = len(m)
    acc = np.empty((n, 3)); phi = np.empty(n); dom = np.empty((n, 3))
    U = C.c_double(); Om = C.c_double()
    _check(lib().orc_force_tree(n, pm, pp, pX, pr, C.byref(p), _d(acc)[1], _d(phi)[1], C.byref(U),
                                C.byref(Om), _d(dom)[1]), "force")
    return acc, phi, U.value, Om.value, dom


def build_state(m, x, v):
    m, pm = _d(m)
    x, px = _d(x)
    v, pv = _d(v)
    n = len(m)
    parent, pp = _i(np.empty(n, dtype=np.int32))
    X = np.empty((n, 3)); V = np.empty((n, 3)); scal = np.empty(9)
    _check(lib().orc_build_state(n, pm, px, pv, pp, _d(X)[1], _d(V)[1], _d(scal)[1]), "build_state")
    return parent, X, V, scal


def to_cartesian(m, parent, X, V, scal):
    m, pm = _d(m)
    parent, pp = _i(parent)
    n = len(m)
    x = np.empty((n, 3)); v = np.empty((n, 3))
    _check(lib().orc_state_to_cartesian(n, pm, pp, _d(X)[1], _d(V)[1], _d(scal)[1], _d(x)[1], _d(v)[1]),
           "to_cartesian")
    return x, v


def leapfrog(m, parent, X, V, scal, H, nsub, p: Params | None = None):
    """One leapfrog division (returns new X, V, scal, force-eval count)."""
    p = p or params()
    m, pm = _d(m)
    parent, pp = _i(parent)
    X = np.array(X, dtype=np.float64, order="C"); V = np.array(V, dtype=np.float64, order="C")
    scal = np.array(scal, dtype=np.float64)
    nf = C.c_int64(0)
    _check(lib().orc_leapfrog(len(m), pm, pp, _d(X)[1], _d(V)[1], _d(scal)[1], C.byref(p), float(H),
                              int(nsub), C.byref(nf)), "leapfrog")
    return X, V, scal, nf.value


def gbs_step(m, parent, X, V, scal, H, p: Params | None = None):
    """One GBS step: returns (X, V, scal, accepted, eps, h_next, force_evals)."""
    p = p or params()
    m, pm = _d(m)
    parent, pp = _i(parent)
    X = np.array(X, dtype=np.float64, order="C"); V = np.array(V, dtype=np.float64, order="C")
    scal = np.array(scal, dtype=np.float64)
    acc = C.c_int32(); eps = C.c_double(); hn = C.c_double(); nf = C.c_int64(0)
    _check(lib().orc_gbs_step(len(m), pm, pp, _d(X)[1], _d(V)[1], _d(scal)[1], C.byref(p), float(H),
                              C.byref(acc), C.byref(eps), C.byref(hn), C.byref(nf)), "gbs_step")
    return X, V, scal, bool(acc.value), eps.value, hn.value, nf.value


def neville(tab):
    """Diagonal T_{k,k} of the Aitken-Neville tableau for rows tab[k] from
    divisions n_k = 2(k+1)."""
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    kf, L = tab.shape
    diag = np.empty_like(tab)
    _check(lib().orc_neville_export(kf, L, _d(tab)[1], _d(diag)[1]), "neville")
    return diag


def integrate(m, x, v, t0, t_end, p: Params | None = None, raise_on_error=True):
    """Full integration (Sec. 2.4 driver).  Returns (x, v, rc, stats dict)."""
    p = p or params()
    m, pm = _d(m)
    x = np.array(x, dtype=np.float64, order="C"); v = np.array(v, dtype=np.float64, order="C")
    st = Stats()
    rc = lib().orc_integrate(len(m), pm, _d(x)[1], _d(v)[1], float(t0), float(t_end), C.byref(p), C.byref(st))
    if raise_on_error and rc < 0:
        raise RuntimeError(f"oracle integrate failed with code {rc}")
    return x, v, rc, st.as_dict()


def _ext_args(g, points):
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(3))
    pts = np.zeros((0, 5)) if points is None else np.asarray(points, dtype=np.float64).reshape(-1, 5)
    pts = np.ascontiguousarray(pts)
    return g, pts


def integrate_ext(m, x, v, t0, t_end, g=(0.0, 0.0, 0.0), points=None, p: Params | None = None,
                  raise_on_error=True):
    """Integration under an external perturbation (Sec. 2.1): a uniform
    acceleration g and fixed Plummer-softened point masses points[k] =
    (M, X, Y, Z, b).  Returns (x, v, rc, stats dict)."""
    p = p or params()
    m, pm = _d(m)
    g, pts = _ext_args(g, points)
    x = np.array(x, dtype=np.float64, order="C"); v = np.array(v, dtype=np.float64, order="C")
    st = Stats()
    rc = lib().orc_integrate_ext(len(m), pm, _d(x)[1], _d(v)[1], float(t0), float(t_end), C.byref(p),
                                 len(pts), _d(g)[1], _d(pts)[1], C.byref(st))
    if raise_on_error and rc < 0:
        raise RuntimeError(f"oracle integrate_ext failed with code {rc}")
    return x, v, rc, st.as_dict()


def external_accel(r, g=(0.0, 0.0, 0.0), points=None, G=1.0):
    """The external acceleration field at positions r[n][3]."""
    g, pts = _ext_args(g, points)
    r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(-1, 3))
    f = np.empty_like(r)
    _check(lib().orc_external_accel(len(pts), _d(g)[1], _d(pts)[1], float(G), len(r), _d(r)[1], _d(f)[1]),
           "external_accel")
    return f


def diagnostics(m, x, v, G=1.0):
    """(E, T, U, P[3], L[3]) with compensated sums."""
    m, pm = _d(m)
    x, px = _d(x)
    v, pv = _d(v)
    out = np.empty(9)
    lib().orc_diagnostics(len(m), pm, px, pv, float(G), _d(out)[1])
    return dict(E=out[0], T=out[1], U=out[2], P=out[3:6].copy(), L=out[6:9].copy())


def sdiv(k_fix, n_div):
    """Division speed-up of the greedy grouping (Sec. 4.2) and the group of each division."""
    g = np.empty(k_fix, dtype=np.int32)
    s = lib().orc_sdiv(int(k_fix), int(n_div), g.ctypes.data_as(C.POINTER(C.c_int32)))
    return s, g


# ---------------------------------------------------------------- replay / TLM
def integrate_rec(m, x, v, t0, t_end, max_accepted, p: Params | None = None):
    """integrate() that also records its accepted steps (fictitious step H_k and
    the MST parent array used) and stops after max_accepted of them.
    Returns (x, v, rc, stats, H[k], parents[k, n])."""
    p = p or params()
    m, pm = _d(m)
    n = len(m)
    x = np.array(x, dtype=np.float64, order="C"); v = np.array(v, dtype=np.float64, order="C")
    H = np.zeros(int(max_accepted))
    par = np.zeros((int(max_accepted), n), dtype=np.int32)
    k = C.c_int64()
    st = Stats()
    rc = lib().orc_integrate_rec(n, pm, _d(x)[1], _d(v)[1], float(t0), float(t_end), C.byref(p), C.byref(st),
                                 int(max_accepted), _d(H)[1], par.ctypes.data_as(C.POINTER(C.c_int32)),
                                 C.byref(k))
    _check(rc if rc < 0 else 0, "integrate_rec")
    return x, v, rc, st.as_dict(), H[:k.value].copy(), par[:k.value].copy()


def replay(m, x, v, t0, H, parents, p: Params | None = None, times=False):
    """Frozen-controller replay in MST coordinates: (x, v, t) after len(H) steps.
    parents None: the driver's own MST builds and rebuilds.  times=True adds
    the time after every step: (x, v, t, t_steps)."""
    p = p or params()
    m, pm = _d(m)
    x = np.array(x, dtype=np.float64, order="C"); v = np.array(v, dtype=np.float64, order="C")
    H = np.ascontiguousarray(H, dtype=np.float64)
    if parents is None:
        pp = None
    else:
        par = np.ascontiguousarray(parents, dtype=np.int32)
        assert par.shape == (len(H), len(m))
        pp = par.ctypes.data_as(C.POINTER(C.c_int32))
    t = C.c_double()
    ts = np.zeros(len(H)) if times else None
    _check(lib().orc_replay(len(m), pm, _d(x)[1], _d(v)[1], float(t0), len(H), _d(H)[1], pp, C.byref(p),
                            C.byref(t), _d(ts)[1] if times else None), "replay")
    return (x, v, t.value, ts) if times else (x, v, t.value)


def rebuild_state(m, parent, X, V, scal, p: Params | None = None):
    """The driver's rebuild (Sec. 3.5) of the state (parent, X, V, scal):
    (new parent, new X, new V, changed)."""
    p = p or params()
    m, pm = _d(m)
    parent = np.array(parent, dtype=np.int32)
    X = np.array(X, dtype=np.float64, order="C"); V = np.array(V, dtype=np.float64, order="C")
    ch = np.zeros(1, dtype=np.int32)
    _check(lib().orc_rebuild_state(len(m), pm, parent.ctypes.data_as(C.POINTER(C.c_int32)), _d(X)[1], _d(V)[1],
                                   _d(scal)[1], C.byref(p), ch.ctypes.data_as(C.POINTER(C.c_int32))),
           "rebuild_state")
    return parent, X, V, bool(ch[0])


def force_tlm(m, r, dr, G=1.0, nthreads=0):
    """Cartesian force, U and their tangents along directions dr [nd, n, 3]:
    (a, U, da [nd, n, 3], dU [nd])."""
    m, pm = _d(m)
    r, pr = _d(r)
    dr = np.ascontiguousarray(dr, dtype=np.float64).reshape(-1, len(m), 3)
    nd = dr.shape[0]
    a = np.empty((len(m), 3)); U = C.c_double()
    da = np.empty_like(dr); dU = np.empty(nd)
    _check(lib().orc_force_tlm(len(m), pm, pr, float(G), nd, _d(dr)[1], _d(a)[1], C.byref(U), _d(da)[1],
                               _d(dU)[1], int(nthreads)), "force_tlm")
    return a, U.value, da, dU


def lagrange_weights(k_fix):
    c = np.empty(k_fix)
    lib().orc_lagrange_weights(int(k_fix), _d(c)[1])
    return c


def replay_tlm(m, x, v, t0, H, dx, dv, p: Params | None = None):
    """Tangent-linear model of the replay (Cartesian form): end state (x, v, t)
    and its tangents (dx, dv [nd, n, 3], dt [nd]) along (dx, dv)."""
    p = p or params()
    m, pm = _d(m)
    n = len(m)
    x = np.array(x, dtype=np.float64, order="C"); v = np.array(v, dtype=np.float64, order="C")
    dx = np.array(dx, dtype=np.float64, order="C").reshape(-1, n, 3)
    dv = np.array(dv, dtype=np.float64, order="C").reshape(-1, n, 3)
    nd = dx.shape[0]
    assert dv.shape == dx.shape
    H = np.ascontiguousarray(H, dtype=np.float64)
    dt = np.zeros(max(nd, 1))
    t = C.c_double()
    _check(lib().orc_replay_tlm(n, pm, _d(x)[1], _d(v)[1], float(t0), len(H), _d(H)[1], C.byref(p), nd,
                                _d(dx)[1], _d(dv)[1], _d(dt)[1], C.byref(t)), "replay_tlm")
    return x, v, t.value, dx, dv, dt[:nd]
