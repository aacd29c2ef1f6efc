"""Pins of the oracle's frozen-controller replay and tangent-linear model (TLM),
the references of the GPU adjoint.

* The replay in MST coordinates repeats a recorded integration bit for bit.
* The Cartesian force tangent equals central differences of the oracle's
  MST force routine (a different code path) and, for two bodies, the
  textbook tidal tensor.
* The Cartesian TLM of the replay equals central differences of the MST
  replay (the method's own map with the recorded steps and topologies), is
  linear in the direction, and its primal end state is the replay's.
* The extrapolation weights are the Neville-Aitken tableau applied to unit
  data and reproduce polynomials in h^2 exactly.
"""
import numpy as np
import pytest

import ics


def _edges(parent, x):
    X = np.zeros_like(x)
    for u, q in enumerate(parent):
        if q >= 0:
            X[u] = x[u] - x[q]
    return X


def _rec(orc, m, x, v, t_end, k, **kw):
    p = orc.params(eta=1e-12, **kw)
    xs, vs, rc, st, H, par = orc.integrate_rec(m, x, v, 0.0, t_end, k, p)
    assert rc == 0
    return xs, vs, st, H, par, p


def test_replay_repeats_integration_bitwise(orc):
    m, x, v = ics.plummer(24, 11)
    xs, vs, st, H, par, p = _rec(orc, m, x, v, 0.3, 200)
    assert st["topo_changes"] > 0          # the record crosses MST topology changes
    xr, vr, tr = orc.replay(m, x, v, 0.0, H, par, p)
    assert np.array_equal(xr, xs) and np.array_equal(vr, vs) and tr == st["t_reached"]


def test_record_stops_after_max_accepted(orc):
    m, x, v = ics.plummer(16, 5)
    xs, vs, st, H, par, p = _rec(orc, m, x, v, 10.0, 7)
    assert st["steps_accepted"] == 7 and len(H) == 7 and st["t_reached"] < 10.0
    xr, vr, tr = orc.replay(m, x, v, 0.0, H, par, p)
    assert np.array_equal(xr, xs) and tr == st["t_reached"]


def test_force_tangent_vs_differences_of_mst_force(orc):
    m, x, v = ics.plummer(40, 3)
    rng = np.random.default_rng(4)
    dr = rng.standard_normal((3, 40, 3))
    a, U, da, dU = orc.force_tlm(m, x, dr)
    p = orc.params(n_d=0)
    parent, X, V, scal = orc.build_state(m, x, v)
    h = 1e-6
    for q in range(3):
        ap, _, Up, _, _ = orc.force(m, parent, _edges(parent, x + h * dr[q]), x + h * dr[q], p)
        am, _, Um, _, _ = orc.force(m, parent, _edges(parent, x - h * dr[q]), x - h * dr[q], p)
        fd = (ap - am) / (2 * h)
        assert np.abs(fd - da[q]).max() <= 1e-7 * np.abs(da[q]).max()
        assert abs((Up - Um) / (2 * h) - dU[q]) <= 1e-7 * abs(dU[q])
    a0, _, U0, _, _ = orc.force(m, parent, X, x, p)
    assert np.abs(a0 - a).max() <= 1e-13 * np.abs(a).max() and abs(U0 - U) <= 1e-14 * U


def test_force_tangent_two_body_tidal_tensor(orc):
    m = np.array([0.7, 1.3])
    x = np.array([[0.1, -0.2, 0.3], [0.9, 0.4, -0.5]])
    e = np.array([[[0.3, -1.0, 0.2], [-0.4, 0.5, 0.9]]])
    a, U, da, dU = orc.force_tlm(m, x, e, G=2.0)
    d = x[1] - x[0]
    r = np.linalg.norm(d)
    T = (np.eye(3) - 3.0 * np.outer(d, d) / r ** 2) / r ** 3
    w = e[0, 1] - e[0, 0]
    assert np.allclose(da[0, 0], 2.0 * m[1] * T @ w, rtol=1e-14, atol=1e-14)
    assert np.allclose(da[0, 1], -2.0 * m[0] * T @ w, rtol=1e-14, atol=1e-14)
    assert np.isclose(dU[0], -2.0 * m[0] * m[1] * d @ w / r ** 3, rtol=1e-14)


@pytest.mark.parametrize("case", ["plummer16", "kepler"])
def test_replay_tlm_vs_differences_of_mst_replay(orc, case):
    if case == "kepler":
        m, x, v = ics.kepler_two_body(0.6, 0.4, 1.0, 0.7, seed=2)
        t_end = 5.0
    else:
        m, x, v = ics.plummer(16, 5)
        t_end = 0.2
    xs, vs, st, H, par, p = _rec(orc, m, x, v, t_end, 60)
    rng = np.random.default_rng(9)
    n = len(m)
    dx = rng.standard_normal((3, n, 3))
    dv = rng.standard_normal((3, n, 3))
    xt, vt, tt, Dx, Dv, Dt = orc.replay_tlm(m, x, v, 0.0, H, dx, dv, p)
    # same map: the Cartesian primal is the MST replay up to rounding
    assert np.abs(xt - xs).max() <= 1e-11 * np.abs(xs).max()
    assert abs(tt - st["t_reached"]) <= 1e-13 * t_end
    h = 1e-6
    for q in range(3):
        xp, vp, tp = orc.replay(m, x + h * dx[q], v + h * dv[q], 0.0, H, par, p)
        xm, vm, tm = orc.replay(m, x - h * dx[q], v - h * dv[q], 0.0, H, par, p)
        assert np.abs((xp - xm) / (2 * h) - Dx[q]).max() <= 1e-6 * np.abs(Dx[q]).max()
        assert np.abs((vp - vm) / (2 * h) - Dv[q]).max() <= 1e-6 * np.abs(Dv[q]).max()
        assert abs((tp - tm) / (2 * h) - Dt[q]) <= 1e-6 * abs(Dt[q]) + 1e-12


def test_replay_tlm_is_linear(orc):
    m, x, v = ics.plummer(12, 7)
    xs, vs, st, H, par, p = _rec(orc, m, x, v, 0.1, 30)
    rng = np.random.default_rng(1)
    d1x, d1v, d2x, d2v = (rng.standard_normal((1, 12, 3)) for _ in range(4))
    _, _, _, A, Av, At = orc.replay_tlm(m, x, v, 0.0, H, d1x, d1v, p)
    _, _, _, B, Bv, Bt = orc.replay_tlm(m, x, v, 0.0, H, d2x, d2v, p)
    _, _, _, Cc, Cv, Ct = orc.replay_tlm(m, x, v, 0.0, H, d1x + 2 * d2x, d1v + 2 * d2v, p)
    assert np.abs(Cc - (A + 2 * B)).max() <= 1e-12 * np.abs(Cc).max()
    assert np.abs(Cv - (Av + 2 * Bv)).max() <= 1e-12 * np.abs(Cv).max()


@pytest.mark.parametrize("kf", [2, 4, 8])
def test_lagrange_weights(orc, kf):
    c = orc.lagrange_weights(kf)
    assert abs(c.sum() - 1.0) <= 1e-13 * np.abs(c).sum()
    tab = np.eye(kf)
    diag = orc.neville(tab)
    assert np.allclose(diag[kf - 1], c, rtol=1e-12, atol=1e-15)
    n = 2.0 * np.arange(1, kf + 1)
    for deg in range(kf):
        assert abs(c @ (1.0 / n ** 2) ** deg - (1.0 if deg == 0 else 0.0)) <= 1e-12 * np.abs(c).sum()


def test_replay_with_own_trees_repeats_integration(orc):
    """Replay without recorded trees (the driver's own MST build and rebuilds,
    Sec. 3.5) and the recorded step lengths repeats the integration bit for
    bit, including the end-time clip's last step: the oracle side of the
    batched systems' replay-mode parity."""
    import ics
    for n, seed, t_end in ((24, 9, 0.3), (5, 2, 0.05)):
        m, x, v = ics.plummer(n, seed)
        xs, vs, rc, st, H, par = orc.integrate_rec(m, x, v, 0.0, t_end, 1000, orc.params(eta=1e-12))
        assert rc == 0 and st["t_reached"] == t_end
        xa, va, ta = orc.replay(m, x, v, 0.0, H, None, orc.params(eta=1e-12))
        assert np.array_equal(xa, xs) and np.array_equal(va, vs) and ta == st["t_reached"]


def test_replay_step_times_are_the_prefix_replays(orc):
    """The per-step times of a replay are the end times of the replays of
    its prefixes, bit for bit (not monotonic at the end: the end-time clip
    of Sec. 2.4 may step back after an overshoot)."""
    m, x, v = ics.plummer(16, 5)
    xs, vs, st, H, par, p = _rec(orc, m, x, v, 0.2, 60)
    xr, vr, tr, ts = orc.replay(m, x, v, 0.0, H, None, p, times=True)
    assert len(ts) == len(H) and ts[-1] == tr and np.all(np.diff(ts[:-3]) > 0)
    for k in (1, len(H) // 3, len(H) - 1):
        assert orc.replay(m, x, v, 0.0, H[:k], None, p)[2] == ts[k - 1]
