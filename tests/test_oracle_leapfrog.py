"""Oracle pins for the regularised leapfrog (paper Sec. 2.1-2.3)."""
import math

import numpy as np
import pytest

import ics
from tests import kepler


def _state(orc, m, x, v, p=None):
    parent, X, V, scal = orc.build_state(m, x, v)
    rho = orc.deconstruct(parent, X)
    acc, phi, U, Om, _ = orc.force(m, parent, X, rho, p)
    vt = v - (m[:, None] * v).sum(0) / m.sum()
    T = 0.5 * (m * (vt ** 2).sum(1)).sum()
    scal[1] = U - T                     # B = -H
    scal[2] = Om
    return parent, X, V, scal


@pytest.mark.parametrize("H,nsub", [(0.05, 1), (0.8, 3), (3.0, 2), (7.0, 5)])
def test_two_body_logh_exact_orbit(orc, H, nsub):
    """Sec. 2.1: with (1,0,0) the leapfrog keeps a Kepler binary exactly on its
    orbit for any step; E, L and the LRL vector are conserved to rounding."""
    m, x, v = ics.kepler_two_body(0.3, 0.7, 1.0, 0.9, seed=4)
    parent, X, V, scal = _state(orc, m, x, v)
    mu = m.sum()
    e0 = kepler.elements(mu, x[1] - x[0], v[1] - v[0])
    X1, V1, s1, nf = orc.leapfrog(m, parent, X, V, scal, H, nsub)
    x1, v1 = orc.to_cartesian(m, parent, X1, V1, s1)
    e1 = kepler.elements(mu, x1[1] - x1[0], v1[1] - v1[0])
    assert nf == nsub
    assert abs(e1["energy"] / e0["energy"] - 1) < 1e-13
    assert np.abs(e1["h"] - e0["h"]).max() < 1e-13 * np.linalg.norm(e0["h"])
    assert np.abs(e1["A"] - e0["A"]).max() < 1e-12 * mu
    assert s1[0] > 0  # time advanced
    # the state moved along the orbit (not trivially unchanged)
    assert np.abs(x1 - x).max() > 1e-3


def test_time_symmetry(orc):
    """Sec. 2.3: the leapfrog is time symmetric: L(-H) L(H) = identity."""
    m, x, v = ics.plummer(8, 12)
    parent, X, V, scal = _state(orc, m, x, v)
    X1, V1, s1, _ = orc.leapfrog(m, parent, X, V, scal, 0.2, 4)
    X2, V2, s2, _ = orc.leapfrog(m, parent, X1, V1, s1, -0.2, 4)
    assert np.abs(X2 - X).max() < 1e-14 * np.abs(X).max() * 50
    assert np.abs(V2 - V).max() < 1e-14 * np.abs(V).max() * 50
    assert abs(s2[0]) < 1e-15


def test_second_order(orc):
    """Sec. 2.3: the leapfrog error has only even powers of h: halving h cuts
    the end-state error by ~4."""
    m, x, v = ics.plummer(6, 13)
    parent, X, V, scal = _state(orc, m, x, v)
    H = 0.05
    ref = orc.leapfrog(m, parent, X, V, scal, H, 512)
    errs = []
    for n in (4, 8, 16):
        Xn, Vn, _, _ = orc.leapfrog(m, parent, X, V, scal, H, n)
        errs.append(np.abs(Vn - ref[1]).max())
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_triplet_001_is_plain_leapfrog(orc):
    """Sec. 2.1: the triplet (0,0,1) is the ordinary leapfrog (dt = ds).  Compare
    with an independent Cartesian drift-kick-drift Stoermer-Verlet."""
    m, x, v = ics.plummer(7, 14)
    p = orc.params(alpha=0.0, beta=0.0, gamma=1.0)
    parent, X, V, scal = _state(orc, m, x, v, p)
    h, n = 0.01, 10
    X1, V1, s1, _ = orc.leapfrog(m, parent, X, V, scal, h * n, n, p)
    x1, v1 = orc.to_cartesian(m, parent, X1, V1, s1)

    def acc(xx):
        d = xx[None, :, :] - xx[:, None, :]
        r2 = (d ** 2).sum(-1)
        np.fill_diagonal(r2, 1.0)
        w = m[None, :] / r2 ** 1.5
        np.fill_diagonal(w, 0.0)
        return (w[:, :, None] * d).sum(1)

    xr, vr = x.copy(), v.copy()
    xr = xr + 0.5 * h * vr
    for k in range(n):
        vr = vr + h * acc(xr)
        xr = xr + (h if k < n - 1 else 0.5 * h) * vr
    assert abs(s1[0] - h * n) < 1e-15
    np.testing.assert_allclose(x1, xr, rtol=0, atol=1e-13)
    np.testing.assert_allclose(v1, vr, rtol=0, atol=1e-13)


def test_force_eval_count(orc):
    """Sec. 4.1: a leapfrog with n substeps costs n force evaluations; a GBS step
    sum_k n_k = k_fix (k_fix + 1), plus one at the start state."""
    m, x, v = ics.plummer(5, 15)
    parent, X, V, scal = _state(orc, m, x, v)
    for n in (1, 2, 7):
        assert orc.leapfrog(m, parent, X, V, scal, 0.01, n)[3] == n
    for kf in (2, 5, 8):
        out = orc.gbs_step(m, parent, X, V, scal, 0.01, orc.params(k_fix=kf, eta=1.0))
        assert out[6] == kf * (kf + 1) + 1
