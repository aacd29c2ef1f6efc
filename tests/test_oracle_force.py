"""Oracle pins for the force loop (paper Sec. 2.1): closed forms, symmetry,
momentum balance and an extended-precision brute force."""
import math

import numpy as np
import pytest


def star_tree(n):
    parent = np.zeros(n, dtype=np.int32)
    parent[0] = -1
    return parent


def cart_state(x, parent):
    X = x - x[np.maximum(parent, 0)]
    X[parent < 0] = 0
    return X


def test_two_body_closed_form(orc):
    m = np.array([2.0, 3.0])
    x = np.array([[0.1, -0.2, 0.3], [1.4, 0.7, -0.9]])
    parent = np.array([-1, 0], dtype=np.int32)
    for G in (1.0, 0.5):
        p = orc.params(G=G)
        acc, phi, U, _, _ = orc.force(m, parent, cart_state(x, parent), x - x[0], p)
        d = x[1] - x[0]
        r = math.sqrt(d @ d)
        np.testing.assert_allclose(acc[0], G * m[1] * d / r ** 3, rtol=2e-16 * 8)
        np.testing.assert_allclose(acc[1], -G * m[0] * d / r ** 3, rtol=2e-16 * 8)
        assert abs(U - G * m[0] * m[1] / r) <= 4e-16 * U


@pytest.mark.parametrize("n", [3, 5, 8, 13])
def test_regular_polygon_closed_form(orc, n):
    """Equal masses on a regular n-gon of radius R: the force on each body is
    central with |a| = G m /(4 R^2) sum_k csc(pi k/n) and
    U = n G m^2/(4 R) sum_k csc(pi k/n)."""
    R, mass = 1.7, 0.3
    ang = 2 * math.pi * np.arange(n) / n
    x = np.stack([R * np.cos(ang), R * np.sin(ang), np.zeros(n)], 1)
    m = np.full(n, mass)
    S = sum(1 / math.sin(math.pi * k / n) for k in range(1, n))
    parent = star_tree(n)
    acc, phi, U, _, _ = orc.force(m, parent, cart_state(x, parent), x - x[0], orc.params(n_d=0))
    amag = mass / (4 * R * R) * S
    for i in range(n):
        np.testing.assert_allclose(acc[i], -amag * x[i] / R, rtol=1e-14, atol=1e-14 * amag)
    assert abs(U - n * mass * mass / (4 * R) * S) <= 1e-14 * U


def test_octahedron_closed_form(orc):
    """Six equal masses at +-R on the axes: |a| = G m/R^2 (1/4 + sqrt(2))."""
    R, mass = 0.8, 1.3
    x = np.array([[R, 0, 0], [-R, 0, 0], [0, R, 0], [0, -R, 0], [0, 0, R], [0, 0, -R]])
    m = np.full(6, mass)
    parent = star_tree(6)
    acc, phi, U, _, _ = orc.force(m, parent, cart_state(x, parent), x - x[0], orc.params(n_d=0))
    amag = mass / R ** 2 * (0.25 + math.sqrt(2))
    for i in range(6):
        np.testing.assert_allclose(acc[i], -amag * x[i] / R, rtol=1e-14, atol=1e-14 * amag)
    assert abs(U - mass * mass / R * (3 * 0.5 + 12 / math.sqrt(2))) <= 1e-14 * U


def _longdouble_force(m, x):
    ml = m.astype(np.longdouble)
    xl = x.astype(np.longdouble)
    n = len(m)
    acc = np.zeros((n, 3), dtype=np.longdouble)
    U = np.longdouble(0)
    for i in range(n):
        d = xl - xl[i]
        r2 = (d * d).sum(1)
        r2[i] = 1
        rinv = 1 / np.sqrt(r2)
        rinv[i] = 0
        acc[i] = ((ml * rinv ** 3)[:, None] * d).sum(0)
        U += ml[i] * (ml * rinv).sum() / 2
    return acc, U


@pytest.mark.parametrize("n,seed", [(16, 1), (64, 2)])
def test_extended_precision_brute_force(orc, n, seed):
    """Normalised error max_i |a_i - a_i^ref| / sum_j m_j/r_ij^2 and |dU/U|
    against an 80-bit long-double brute force, with MST coordinates."""
    import ics
    m, x, _ = ics.plummer(n, seed)
    parent, X, V, scal = orc.build_state(m, x, np.zeros_like(x))
    rho = orc.deconstruct(parent, X)
    acc, phi, U, _, _ = orc.force(m, parent, X, rho)
    ref, Uref = _longdouble_force(m, rho)
    for i in range(n):
        d = rho - rho[i]
        r2 = (d * d).sum(1); r2[i] = np.inf
        scale = (m / r2).sum()
        assert float(np.abs(acc[i] - ref[i]).max()) / scale < 1e-14
    assert abs(float((U - Uref) / Uref)) < 1e-15


def test_momentum_balance(orc):
    import ics
    m, x, _ = ics.plummer(200, 3)
    parent, X, V, scal = orc.build_state(m, x, np.zeros_like(x))
    rho = orc.deconstruct(parent, X)
    acc, phi, U, _, _ = orc.force(m, parent, X, rho)
    tot = (m[:, None] * acc).sum(0)
    terms = 0.0
    for i in range(200):
        d = rho - rho[i]
        r2 = (d * d).sum(1); r2[i] = np.inf
        terms += m[i] * (m / r2).sum()
    assert np.abs(tot).max() < 200 * np.finfo(float).eps * terms


def test_phi_and_U_consistent(orc):
    import ics
    m, x, _ = ics.plummer(50, 4)
    parent, X, V, scal = orc.build_state(m, x, np.zeros_like(x))
    rho = orc.deconstruct(parent, X)
    for G in (1.0, 2.5):
        acc, phi, U, _, _ = orc.force(m, parent, X, rho, orc.params(G=G))
        assert abs(U - 0.5 * G * (m * phi).sum()) < 1e-14 * U


def test_omega_and_gradient(orc):
    """TTL Omega with omega_mass_max (READING: only bodies with m <= threshold
    couple): Omega equals the force function of the light subset, and dOmega is
    its gradient (checked by central differences)."""
    rng = np.random.default_rng(9)
    n = 12
    m = np.where(np.arange(n) < 4, 1.0, 1e-3)
    x = rng.standard_normal((n, 3))
    parent = star_tree(n)
    p = orc.params(beta=1.0, omega_mass_max=1e-2, n_d=0)
    acc, phi, U, Om, dOm = orc.force(m, parent, cart_state(x, parent), x - x[0], p)
    light = m <= 1e-2
    ml, xl = m[light], x[light]
    Omref = sum(ml[i] * ml[j] / np.linalg.norm(xl[i] - xl[j]) for i in range(len(ml)) for j in range(i + 1, len(ml)))
    assert abs(Om - Omref) < 1e-14 * Omref
    h = 1e-6
    for i in [5, 9]:
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h; xm[i, c] -= h
            Op = orc.force(m, parent, cart_state(xp, parent), xp - xp[0], p)[3]
            Omn = orc.force(m, parent, cart_state(xm, parent), xm - xm[0], p)[3]
            assert abs((Op - Omn) / (2 * h) - dOm[i, c]) < 1e-7 * np.abs(dOm).max()
    assert np.all(dOm[~light] == 0)
