"""Pins of the oracle's earliest-k acceptance (accept_rule 1: eq. gbs-criterion
judged at every k = 2..k_fix as in the serial scheme of Sec. 2.3, against the
fixed k_fix of Sec. 4.2).

* With a tolerance every order passes (eta = 1), the step returns T_22, the
  first Richardson combination of the n = 2 and n = 4 leapfrogs,
  L4 + (L4 - L2) / 3, formed here from the oracle's single-leapfrog entry
  point; the next step follows eq. hnext with k = 2, exponent 1/3.
* With eta between the error measures of two orders, the accepted order is
  the first one below eta: its result's true error (the closed-form LogH
  two-body flow) lies below eta's scale, and the step differs from the
  k_fix = 8 result.
* With eta below every eps_k for k < k_fix the two rules agree bit for bit.
"""
import math

import numpy as np

from tests.test_oracle_gbs_error import _kepler_exact_after, _two_body, _with_binding_energy


def test_eta_one_returns_richardson_of_two_leapfrogs(orc):
    m, x, v = _two_body(0.6, 1.0, 3)
    parent, X, V, scal, U0 = _with_binding_energy(orc, m, x, v)
    H = 0.05
    X1, V1, s1, acc, eps, hn, _ = orc.gbs_step(m, parent, X, V, scal, H, orc.params(eta=1.0, accept_rule=1))
    assert acc
    X2, V2, s2, _ = orc.leapfrog(m, parent, X, V, scal, H, 2)
    X4, V4, s4, _ = orc.leapfrog(m, parent, X, V, scal, H, 4)
    want_X = X4 + (X4 - X2) / 3.0
    want_V = V4 + (V4 - V2) / 3.0
    want_t = s4[0] + (s4[0] - s2[0]) / 3.0
    np.testing.assert_allclose(X1, want_X, rtol=0, atol=1e-14 * np.abs(X).max())
    np.testing.assert_allclose(V1, want_V, rtol=0, atol=1e-14 * np.abs(V).max())
    assert abs(s1[0] - want_t) <= 1e-14 * abs(want_t)
    p = orc.params()
    f = min(max(p.a_gbs * (1.0 / max(eps, 1e-300)) ** (1.0 / 3.0), p.f_min), p.f_max)
    assert abs(hn - H * f) <= 1e-15 * H * f


def _gbs(orc, m, parent, X, V, scal, H, eta, rule, kf=8):
    return orc.gbs_step(m, parent, X, V, scal, H, orc.params(eta=eta, accept_rule=rule, k_fix=kf))


def test_first_passing_order_is_accepted_kepler(orc):
    """e = 0.5, a step of 4 radians of eccentric anomaly: eps_k falls from
    ~1e-2 (k = 2) to ~1e-8 (k = 8).  For eta between eps_{k-1} and eps_k's
    neighbours the accepted result is T_kk of the first passing order: equal
    to a k_fix = k step, with a closed-form error below eta's scale."""
    m, x, v = _two_body(0.5, math.pi, 5)
    parent, X, V, scal, U0 = _with_binding_energy(orc, m, x, v)
    H = 4.0 * (m[0] * m[1]) / math.sqrt(m.sum())
    eps = {k: _gbs(orc, m, parent, X, V, scal, H, 1.0, 0, kf=k)[4] for k in range(2, 9)}
    r1, v1, dt, _ = _kepler_exact_after(m, x, v, H)
    c = int(np.flatnonzero(parent >= 0)[0])
    sgn = 1.0 if c == 1 else -1.0
    used = 0
    for k in range(3, 8):
        if not (eps[k] < eps[k - 1] and all(eps[j] > eps[k] for j in range(2, k))):
            continue
        eta = math.sqrt(eps[k] * min(eps[j] for j in range(2, k)))   # passes at k, fails below
        Xa, Va, sa, acc, e_a, hn_a, _ = _gbs(orc, m, parent, X, V, scal, H, eta, 1)
        assert acc and e_a == eps[k]
        Xk, Vk, sk, acck, _, _, _ = _gbs(orc, m, parent, X, V, scal, H, 1.0, 0, kf=k)
        assert np.array_equal(Xa, Xk) and np.array_equal(Va, Vk) and np.array_equal(sa, sk)
        # the result's true error is below eta's scale (eps_k bounds T_{k-1,k-1}'s)
        err = np.linalg.norm(sgn * Va[c] - v1) / np.linalg.norm(v1)
        assert err <= 10 * eta, (k, err, eta)
        p = orc.params()
        f = min(max(p.a_gbs * (eta / eps[k]) ** (1.0 / (2 * k - 1)), p.f_min), p.f_max)
        assert abs(hn_a - H * f) <= 1e-14 * H * f
        used += 1
    assert used >= 3, eps


def test_rules_agree_when_only_k_fix_passes(orc):
    m, x, v = _two_body(0.9, 2.0, 7)
    parent, X, V, scal, U0 = _with_binding_energy(orc, m, x, v)
    H = 3.0 * (m[0] * m[1]) / math.sqrt(m.sum())
    eps = {k: _gbs(orc, m, parent, X, V, scal, H, 1.0, 0, kf=k)[4] for k in range(2, 9)}
    eta = 0.5 * (eps[8] + min(eps[k] for k in range(2, 8)))
    assert eps[8] < eta < min(eps[k] for k in range(2, 8))
    a = _gbs(orc, m, parent, X, V, scal, H, eta, 0)
    b = _gbs(orc, m, parent, X, V, scal, H, eta, 1)
    assert a[3] and b[3]
    for u, w in zip(a[:3], b[:3]):
        assert np.array_equal(u, w)
    assert a[4] == b[4] and a[5] == b[5]


def test_rule_one_rejects_when_no_order_passes(orc):
    m, x, v = _two_body(0.9, 0.0, 7)
    parent, X, V, scal, U0 = _with_binding_energy(orc, m, x, v)
    H = 6.0 * (m[0] * m[1]) / math.sqrt(m.sum())
    Xa, Va, sa, acc, eps, hn, _ = _gbs(orc, m, parent, X, V, scal, H, 1e-14, 1)
    assert not acc and hn == 0.5 * H
    assert np.array_equal(Xa, X) and np.array_equal(Va, V)
