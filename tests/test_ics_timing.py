"""The timing-test clusters of Sec. 5.4: Hernquist spheres without hard
binaries, and the unit conversion of their 0.1 Myr integration time."""
import math

import numpy as np
import pytest

import ics


def _hard_brute(m, x, v):
    vc = v - (m[:, None] * v).sum(0) / m.sum()
    th = 0.5 * np.mean(m * (vc * vc).sum(1))
    out = []
    for a in range(len(m)):
        for b in range(a + 1, len(m)):
            d, w = x[b] - x[a], v[b] - v[a]
            mu = m[a] * m[b] / (m[a] + m[b])
            if m[a] * m[b] / math.sqrt(d @ d) - 0.5 * mu * (w @ w) >= th:
                out.append((a, b))
    return out


@pytest.mark.parametrize("n,seed", [(10, 1000), (10, 1001), (10, 4002), (14, 3000), (30, 5), (200, 7)])
def test_hard_binaries_matches_all_pairs(n, seed):
    m, x, v = ics.hernquist(n, seed)
    assert ics.hard_binaries(m, x, v) == _hard_brute(m, x, v)


def test_hard_binary_is_found():
    """A tight pair planted in a cluster is reported, and nothing else."""
    m, x, v = ics.hernquist(100, 3)
    assert ics.hard_binaries(m, x, v) == []
    x = x.copy(); v = v.copy()
    x[7] = x[3] + np.array([1e-4, 0.0, 0.0])
    v[7] = v[3]
    assert ics.hard_binaries(m, x, v) == [(3, 7)]


@pytest.mark.parametrize("n", [10, 21, 379])
def test_timing_clusters_have_no_hard_binaries(n):
    for seed in (1, 2, 3):
        m, x, v, k = ics.timing_cluster(n, seed)
        assert len(m) == n and _hard_brute(m, x, v) == []
        assert abs(m.sum() - 1.0) < 1e-12


def test_timing_sizes():
    """Twenty sizes, logarithmic from 10 to 10^4, including the paper's 264,
    379 and 1129."""
    s = ics.timing_sizes()
    assert len(s) == 20 and s[0] == 10 and s[-1] == 10000
    assert {264, 379, 1129} <= set(s)


def test_timing_time_unit():
    """sqrt(r_half^3 / (G M)) for r_half = 10 pc, M = 1e7 Msun, from G in
    pc (km/s)^2 / Msun and 1 km/s = 1.0227121650537077 pc/Myr."""
    G = 4.300917270e-3 * 1.0227121650537077 ** 2       # pc^3 / (Msun Myr^2)
    tu = math.sqrt(10.0 ** 3 / (G * 1e7))
    assert abs(tu / ics.TIMING_MYR_PER_UNIT - 1) < 1e-6
    assert abs(ics.TIMING_T_END * ics.TIMING_MYR_PER_UNIT - 0.1) < 1e-15
