"""Oracle pins for GBS extrapolation, step control and the driver (paper
Sec. 2.3, 2.4, 4.2, 5.1)."""
import math

import numpy as np
import pytest

import ics
from tests import kepler


def test_neville_reproduces_polynomials(orc):
    """Sec. 4.2: Neville-Aitken polynomial extrapolation in h^2 is exact for
    data that are polynomials of degree < k_fix in h^2 (Deuflhard n_k = 2k)."""
    rng = np.random.default_rng(3)
    for kf in (2, 4, 8):
        c = rng.standard_normal((kf, 5))
        nk = 2 * np.arange(1, kf + 1)
        h2 = (1.0 / nk) ** 2
        tab = np.stack([sum(c[j] * h2[k] ** j for j in range(kf)) for k in range(kf)])
        diag = orc.neville(tab)
        np.testing.assert_allclose(diag[kf - 1], c[0], rtol=0, atol=1e-12 * np.abs(c).max())
        # lower diagonal entries are exact for lower-degree data
        tab2 = np.stack([c[0] + c[1] * h2[k] for k in range(kf)])
        d2 = orc.neville(tab2)
        for k in range(1, kf):
            np.testing.assert_allclose(d2[k], c[0], rtol=0, atol=1e-13 * np.abs(c).max())


def test_neville_first_column_is_richardson(orc):
    """Two divisions (n = 2, 4): T_22 = (4 T_2 - T_1)/3, the classic Richardson
    step for an h^2 error."""
    tab = np.array([[1.0, 2.0], [1.5, 2.5]])
    d = orc.neville(tab)
    np.testing.assert_allclose(d[1], (4 * tab[1] - tab[0]) / 3, rtol=1e-15)


def _three_body(orc):
    m = np.array([1.0, 0.6, 0.3])
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [-0.4, 1.3, 0.2]])
    v = np.array([[0.0, -0.1, 0.0], [0.1, 0.8, 0.05], [-0.6, -0.2, 0.1]])
    parent, X, V, scal = orc.build_state(m, x, v)
    rho = orc.deconstruct(parent, X)
    _, _, U, _, _ = orc.force(m, parent, X, rho)
    vt = v - (m[:, None] * v).sum(0) / m.sum()
    scal[1] = U - 0.5 * (m * (vt ** 2).sum(1)).sum()
    return m, parent, X, V, scal


@pytest.mark.parametrize("kf", [2, 3])
def test_gbs_order(orc, kf):
    """Sec. 2.3: with k divisions the extrapolated step has local error
    O(H^(2k+1)): halving H divides the error by ~2^(2k+1)."""
    m, parent, X, V, scal = _three_body(orc)
    p = orc.params(k_fix=kf, eta=1.0)
    pref = orc.params(k_fix=8, eta=1.0)
    errs = []
    for H in (0.08, 0.04):
        Xa = orc.gbs_step(m, parent, X, V, scal, H, p)[0]
        Xr, Vr, sr = X, V, scal
        for _ in range(8):
            Xr, Vr, sr = orc.gbs_step(m, parent, Xr, Vr, sr, H / 8, pref)[:3]
        errs.append(np.abs(Xa - Xr).max())
    ratio = errs[0] / errs[1]
    want = 2 ** (2 * kf + 1)
    assert 0.6 * want < ratio < 1.6 * want, (errs, ratio)


def test_gbs_accept_reject_and_step_control(orc):
    """eq. gbs-criterion / eq. hnext: a step is accepted iff eps <= eta; after
    acceptance H_next = H * clamp(a_GBS (eta/eps)^(1/(2k-1)), f_min, f_max);
    after rejection the state is unchanged and H is halved."""
    m, parent, X, V, scal = _three_body(orc)
    p = orc.params(k_fix=4, eta=1e-10)
    X1, V1, s1, acc, eps, hn, nf = orc.gbs_step(m, parent, X, V, scal, 0.05, p)
    assert acc and eps <= 1e-10
    f = min(max(0.9 * (1e-10 / eps) ** (1 / 7), 0.1), 4.0)
    assert abs(hn - 0.05 * f) < 1e-15
    X2, V2, s2, acc2, eps2, hn2, _ = orc.gbs_step(m, parent, X, V, scal, 2.0, p)
    assert not acc2 and eps2 > 1e-10 and hn2 == 1.0
    assert np.array_equal(X2, X) and np.array_equal(V2, V) and np.array_equal(s2, scal)


def test_gbs_nonfinite_rejects(orc):
    """A NaN produced inside a step (by a step large enough to pass through a
    collision with the wrong sign of time) must never count as converged."""
    m, parent, X, V, scal = _three_body(orc)
    out = orc.gbs_step(m, parent, X, V, scal, 1e200, orc.params(k_fix=3, eta=1e-6))
    assert not out[3]


@pytest.mark.parametrize("orbits", [0.37, 3.3, 20.7])
def test_kepler_end_state_closed_form(orc, orbits):
    """Sec. 5.1: an e = 0.9 binary integrated with eta = 1e-12 matches the
    analytic Kepler solution at the reached time."""
    m, x, v = ics.kepler_two_body(0.5, 0.5, 1.0, 0.9, seed=3)
    tend = orbits * 2 * math.pi
    x1, v1, rc, st = orc.integrate(m, x, v, 0.0, tend, orc.params(eta=1e-12))
    assert rc == 0
    assert abs(st["t_reached"] - tend) <= 1e-14 * tend
    r, u = kepler.propagate(1.0, x[1] - x[0], v[1] - v[0], st["t_reached"])
    assert np.abs((x1[1] - x1[0]) - r).max() < 5e-12 * np.linalg.norm(r)
    assert np.abs((v1[1] - v1[0]) - u).max() < 5e-12 * np.linalg.norm(u)
    # conserved COM (never kicked)
    np.testing.assert_allclose((m[:, None] * v1).sum(0), 0.0, atol=1e-15)


def test_kepler_invariants_and_lrl(orc):
    """Sec. 5.1: E, L and the Laplace-Runge-Lenz vector of a random-orientation
    e = 0.9 binary; A.L = 0 and e = |A|/(G M) hold for the end state."""
    m, x, v = ics.kepler_two_body(0.5, 0.5, 1.0, 0.9, seed=17)
    x1, v1, rc, st = orc.integrate(m, x, v, 0.0, 10 * 2 * math.pi, orc.params(eta=1e-12))
    el0 = kepler.elements(1.0, x[1] - x[0], v[1] - v[0])
    el1 = kepler.elements(1.0, x1[1] - x1[0], v1[1] - v1[0])
    assert abs(el1["energy"] / el0["energy"] - 1) < 1e-12
    assert np.abs(el1["h"] - el0["h"]).max() < 1e-12 * np.linalg.norm(el0["h"])
    assert abs(el1["A"] @ el1["h"]) < 1e-12
    assert abs(el1["e"] - 0.9) < 1e-12
    cosang = el1["A"] @ el0["A"] / (np.linalg.norm(el1["A"]) * np.linalg.norm(el0["A"]))
    assert math.acos(min(1.0, cosang)) < 1e-10           # theta_LRL drift


def test_plummer_energy_conservation(orc):
    m, x, v = ics.plummer(32, 101)
    d0 = orc.diagnostics(m, x, v)
    x1, v1, rc, st = orc.integrate(m, x, v, 0.0, 0.25, orc.params(eta=1e-12))
    d1 = orc.diagnostics(m, x1, v1)
    assert rc == 0
    assert abs((d1["E"] - d0["E"]) / d0["E"]) < 1e-12
    np.testing.assert_allclose(d1["P"], d0["P"], atol=1e-15)
    np.testing.assert_allclose(d1["L"], d0["L"], atol=1e-13)
    assert st["force_evals"] >= 73 * st["steps_accepted"]


def test_driver_backward_in_time(orc):
    """Negative intervals integrate backwards (time-symmetric leapfrog)."""
    m, x, v = ics.kepler_two_body(0.5, 0.5, 1.0, 0.7, seed=5)
    x1, v1, rc, st = orc.integrate(m, x, v, 0.0, -2.1, orc.params(eta=1e-12))
    assert rc == 0 and abs(st["t_reached"] + 2.1) < 1e-13
    r, u = kepler.propagate(1.0, x[1] - x[0], -(v[1] - v[0]), 2.1)   # reverse velocities
    assert np.abs((x1[1] - x1[0]) - r).max() < 1e-11


def test_first_step_and_halvings(orc):
    """Sec. 2.4: the first step ds = q U dt (clipped to the interval) is far too
    long for a binary with many orbits in the interval; the driver must reject
    and halve until convergence and still reach t_end."""
    m, x, v = ics.kepler_two_body(0.5, 0.5, 1.0, 0.9, seed=8)
    x1, v1, rc, st = orc.integrate(m, x, v, 0.0, 40.0, orc.params(q_first=1.0, eta=1e-10))
    assert rc == 0 and st["steps_rejected"] >= 3 and abs(st["t_reached"] - 40.0) < 1e-13


def test_failure_modes(orc):
    m, x, v = ics.plummer(5, 22)
    _, _, rc, st = orc.integrate(m, x, v, 0.0, 1.0, orc.params(eta=1e-30, max_halvings=3), raise_on_error=False)
    assert rc == orc.E_NOCONV
    x1, v1, rc, st = orc.integrate(m, x, v, 0.0, 10.0, orc.params(max_steps=3), raise_on_error=False)
    assert rc == orc.E_MAXSTEPS and 0 < st["t_reached"] < 10.0 and np.all(np.isfinite(x1))
    xb = x.copy(); xb[3] = xb[1]
    assert orc.integrate(m, xb, v, 0.0, 1.0, raise_on_error=False)[2] == orc.E_COINCIDENT
    xb = x.copy(); xb[2, 1] = np.nan
    assert orc.integrate(m, xb, v, 0.0, 1.0, raise_on_error=False)[2] == orc.E_NONFINITE
    assert orc.integrate(m, x, v, 0.0, 1.0, orc.params(k_fix=1), raise_on_error=False)[2] == orc.E_INVAL
    assert orc.integrate(m[:1], x[:1], v[:1], 0.0, 1.0, raise_on_error=False)[2] == orc.E_INVAL
    mb = m.copy(); mb[0] = 0.0
    assert orc.integrate(mb, x, v, 0.0, 1.0, raise_on_error=False)[2] == orc.E_INVAL


def test_time_tolerance_warning(orc):
    m, x, v = ics.kepler_two_body(0.5, 0.5, 1.0, 0.9, seed=3)
    _, _, rc, st = orc.integrate(m, x, v, 0.0, 3.3 * 2 * math.pi, orc.params(max_time_iter=0),
                                 raise_on_error=False)
    assert rc == orc.W_TIME_TOL and st["time_iters"] == 1


def test_rebuild_keeps_trajectory(orc):
    """Sec. 3.5: rebuilding the MST every step (or never) must not change the
    trajectory beyond rounding-level differences."""
    m, x, v = ics.plummer(24, 31)
    outs = []
    for rb in (1, 1000000):
        x1, v1, rc, st = orc.integrate(m, x, v, 0.0, 0.2, orc.params(eta=1e-13, rebuild_every=rb))
        outs.append((x1, st))
    assert outs[0][1]["topo_changes"] > 0
    assert np.abs(outs[0][0] - outs[1][0]).max() < 1e-10


def test_ttl_triplet_runs_and_conserves(orc):
    """TTL (0,1,0) with Omega over the light bodies (READING of Sec. 2.1)."""
    m, x, v = ics.plummer(10, 41)
    m = m.copy(); m[:3] *= 10
    p = orc.params(alpha=0.0, beta=1.0, gamma=0.0, omega_mass_max=m.min() * 1.5, eta=1e-11)
    d0 = orc.diagnostics(m, x, v)
    x1, v1, rc, st = orc.integrate(m, x, v, 0.0, 0.1, p)
    d1 = orc.diagnostics(m, x1, v1)
    assert rc == 0 and abs((d1["E"] - d0["E"]) / d0["E"]) < 1e-10
