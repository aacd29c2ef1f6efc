"""Synthetic initial conditions: shapes, seeds, centre of mass, virial state."""
import math

import numpy as np

import ics


def _energy(m, x, v):
    d = x[:, None, :] - x[None, :, :]
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    U = 0.5 * (m[:, None] * m[None, :] / r).sum()
    T = 0.5 * (m * (v ** 2).sum(1)).sum()
    return T, U


def test_plummer_henon_units():
    m, x, v = ics.plummer(2000, 11)
    assert m.shape == (2000,) and x.shape == (2000, 3) and v.shape == (2000, 3)
    assert abs(m.sum() - 1.0) < 1e-14
    assert np.abs((m[:, None] * x).sum(0)).max() < 1e-14
    assert np.abs((m[:, None] * v).sum(0)).max() < 1e-14
    T, U = _energy(m, x, v)
    # Henon units: E = -1/4, 2T/U = 1, up to sampling noise at N = 2000
    assert abs((T - U) + 0.25) < 0.03
    assert abs(2 * T / U - 1.0) < 0.08


def test_seed_reproducible_and_distinct():
    a = ics.plummer(64, 5)
    b = ics.plummer(64, 5)
    c = ics.plummer(64, 6)
    for p, q in zip(a, b):
        assert np.array_equal(p, q)
    assert not np.array_equal(a[1], c[1])


def test_embedded_binary_elements():
    m, x, v = ics.plummer_with_binary(100, 3)
    assert len(m) == 102 and m[-1] == m[-2] == 0.005
    r = x[-1] - x[-2]
    u = v[-1] - v[-2]
    mu = 0.01
    eps = 0.5 * u @ u - mu / np.linalg.norm(r)
    a = -mu / (2 * eps)
    h = np.cross(r, u)
    e = np.linalg.norm(np.cross(u, h) / mu - r / np.linalg.norm(r))
    assert abs(a - 1e-3) < 1e-15 and abs(e - 0.9) < 1e-12
    assert abs(np.linalg.norm(r) - 1e-3 * 1.9) < 1e-15   # apocentre


def test_pythagorean_geometry():
    m, x, v = ics.pythagorean()
    d = lambda i, j: np.linalg.norm(x[i] - x[j])
    # each body faces the side equal to its own mass (3, 4, 5)
    assert d(1, 2) == 3.0 and d(0, 2) == 4.0 and d(0, 1) == 5.0
    assert np.allclose((m[:, None] * x).sum(0), 0.0)


def test_lidov_kozai_setup():
    m, x, v = ics.lidov_kozai()
    rin = x[1] - x[0]
    vin = v[1] - v[0]
    hin = np.cross(rin, vin)
    cm_in = (m[0] * x[0] + m[1] * x[1]) / (m[0] + m[1])
    vcm_in = (m[0] * v[0] + m[1] * v[1]) / (m[0] + m[1])
    hout = np.cross(x[2] - cm_in, v[2] - vcm_in)
    inc = math.degrees(math.acos(hin @ hout / np.linalg.norm(hin) / np.linalg.norm(hout)))
    assert abs(inc - 80.0) < 1e-9
    assert np.allclose((m[:, None] * v).sum(0), 0.0, atol=1e-15)


def test_batch_subsystems_layout():
    off, m, x, v = ics.batch_subsystems(300, 9)
    sizes = np.diff(off)
    assert off[0] == 0 and sizes.min() >= 3 and sizes.max() <= 64
    assert (sizes == 3).mean() > 0.05
    for s in range(0, 300, 37):
        o, k = off[s], sizes[s]
        ms = m[o:o + k]
        assert ms[0] == 1.0 and np.all(ms[1:] == 1e-5)
        assert np.abs((ms[:, None] * x[o:o + k]).sum(0)).max() < 1e-15
