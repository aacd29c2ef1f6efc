"""Pins of the oracle's external perturbation (Sec. 2.1: a position-dependent
acceleration f_i added to the Newtonian one, with the binding energy B taking
the work of f analytically over each kick).  The field: a uniform
acceleration g plus fixed Plummer-softened point masses (M, R, b), the
gradient field of Phi(r) = -g.r - G sum M / sqrt(|r - R|^2 + b^2)."""
import numpy as np
import pytest

import ics

G = 1.0


def phi_ext(r, g, points):
    r = np.atleast_2d(r)
    out = -(r @ np.asarray(g, dtype=float))
    for M, X, Y, Z, b in np.atleast_2d(points) if points is not None else []:
        d = r - np.array([X, Y, Z])
        out = out - G * M / np.sqrt((d * d).sum(1) + b * b)
    return out


def test_field_is_minus_grad_phi(orc):
    rng = np.random.default_rng(7)
    pts = np.array([[2.0, 0.3, -0.2, 0.5, 0.1], [0.5, -1.0, 1.0, 0.0, 0.0]])
    g = np.array([0.1, -0.2, 0.05])
    r = rng.standard_normal((20, 3)) * 2.0
    f = orc.external_accel(r, g, pts, G)
    h = 1e-5
    for c in range(3):
        e = np.zeros(3); e[c] = h
        fd = -(phi_ext(r + e, g, pts) - phi_ext(r - e, g, pts)) / (2 * h)
        assert np.abs(fd - f[:, c]).max() <= 1e-7 * np.abs(f).max()


def test_field_closed_form_on_an_axis(orc):
    """One unsoftened mass M = 3 at the origin: f(2, 0, 0) = (-3/4, 0, 0);
    softened by b = 1 at r = (0, 1, 0): f = (0, -3 / 2^(3/2), 0)."""
    f = orc.external_accel([[2.0, 0.0, 0.0]], points=[[3.0, 0.0, 0.0, 0.0, 0.0]])
    assert np.array_equal(f, [[-0.75, 0.0, 0.0]])
    f = orc.external_accel([[0.0, 1.0, 0.0]], g=(0.5, 0.0, 0.0), points=[[3.0, 0.0, 0.0, 0.0, 1.0]])
    assert np.abs(f - [[0.5, -3.0 / 2.0 ** 1.5, 0.0]]).max() <= 1e-15


def _com(m, a):
    return (m[:, None] * a).sum(0) / m.sum()


def test_uniform_field_moves_only_the_centre_of_mass(orc):
    """Equivalence principle: a uniform g leaves the internal motion as it is
    and carries the centre of mass on the parabola r0 + v0 t + g t^2 / 2."""
    m, x, v, _ = ics.workload("plummer32")
    v = v + np.array([0.2, 0.0, -0.1])
    g = np.array([0.3, -0.2, 0.1])
    T = 0.5
    p = orc.params(eta=1e-12)
    x0, v0, rc0, _ = orc.integrate(m, x, v, 0.0, T, p)
    x1, v1, rc1, st = orc.integrate_ext(m, x, v, 0.0, T, g=g, p=p)
    assert rc0 == rc1 == 0 and abs(st["t_reached"] - T) <= 1e-14
    R = np.abs(x0 - _com(m, x0)).max()
    Vs = np.abs(v0 - _com(m, v0)).max()
    assert np.abs((x1 - _com(m, x1)) - (x0 - _com(m, x0))).max() <= 1e-11 * R
    assert np.abs((v1 - _com(m, v1)) - (v0 - _com(m, v0))).max() <= 1e-11 * Vs
    rc, vc = _com(m, x), _com(m, v)
    assert np.abs(_com(m, x1) - (rc + vc * T + 0.5 * g * T * T)).max() <= 1e-13
    assert np.abs(_com(m, v1) - (vc + g * T)).max() <= 1e-13


def _cluster_near_mass():
    """A 32-body Plummer cluster on a near-circular orbit at distance 4 around
    a softened point mass of 5 (b = 0.5): the field's tidal part is strong
    (tidal radius ~1.6), so it does work on the internal motion."""
    m, x, v, _ = ics.workload("plummer32")
    pts = np.array([[5.0, 4.0, 0.0, 0.0, 0.5]])
    vc = np.sqrt(5.0 * 16.0 / (16.0 + 0.25) ** 1.5)
    return m, x, v + np.array([0.0, vc, 0.0]), pts


def test_point_mass_field_conserves_total_energy_and_angular_momentum(orc):
    """In a static field the energy T - U + sum m Phi(r) is conserved; a
    spherical field around R exerts no torque about R, so sum m (r - R) x v is
    conserved too.  The internal energy changes by several per cent, so a
    missing or wrong B update (the work of f) breaks the first."""
    m, x, v, pts = _cluster_near_mass()
    T = 1.0
    x1, v1, rc, st = orc.integrate_ext(m, x, v, 0.0, T, points=pts, p=orc.params(eta=1e-12))
    assert rc == 0 and abs(st["t_reached"] - T) <= 1e-14

    def etot(xx, vv):
        return orc.diagnostics(m, xx, vv)["E"] + float((m * phi_ext(xx, (0, 0, 0), pts)).sum())

    def lz(xx, vv):
        return (m[:, None] * np.cross(xx - pts[0, 1:4], vv)).sum(0)

    e0, e1 = etot(x, v), etot(x1, v1)
    assert abs(e1 / e0 - 1) <= 1e-11, e1 / e0 - 1
    L0, L1 = lz(x, v), lz(x1, v1)
    assert np.abs(L1 - L0).max() <= 1e-11 * np.abs(L0).max()
    # the perturbation really acts: the internal energy moves and the COM turns
    ein0 = orc.diagnostics(m, x - _com(m, x), v - _com(m, v))["E"]
    ein1 = orc.diagnostics(m, x1 - _com(m, x1), v1 - _com(m, v1))["E"]
    assert abs(ein1 / ein0 - 1) > 1e-2
    assert np.linalg.norm(_com(m, v1) - _com(m, v)) > 0.2


def test_no_field_is_the_plain_integration(orc):
    """With g = 0 and no points the perturbed driver takes the plain one's
    path bit for bit (f = 0 adds exact zeros)."""
    m, x, v, _ = ics.workload("plummer32")
    p = orc.params(eta=1e-12)
    a = orc.integrate(m, x, v, 0.0, 0.2, p)
    b = orc.integrate_ext(m, x, v, 0.0, 0.2, p=p)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[3] == b[3]


def test_beta_is_rejected(orc):
    m, x, v, _ = ics.workload("plummer32")
    _, _, rc, _ = orc.integrate_ext(m, x, v, 0.0, 0.1, g=(1.0, 0.0, 0.0), p=orc.params(beta=1.0, alpha=0.0),
                                    raise_on_error=False)
    assert rc < 0
