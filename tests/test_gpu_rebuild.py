"""Coordinate round trips (Sec. 3.5) on the GPU through the C ABI, against the
oracle: the MST and chain built on the GPU, their edge vectors and the
rebuilt Cartesian state.

Tolerances: the structures are built under the same strict edge order from
the same positions, so the mean levels agree exactly; the states differ only
by the summation order of the centre-of-mass sums (compensated on both
sides), so after C cycles they agree to ~C * 1e-16 of the position scale
(bound 1e-13 for 30 cycles).  On a dyadic lattice every operation is exact
and the state must return bit for bit.  With plain centre-of-mass sums in
index order (kinds 2, 3: the paper's test) every operation is the oracle's,
and the GPU repeats its round trips bit for bit."""
import sys

import numpy as np
import pytest

import ics

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_03180_amd as M
    c = M.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def M():
    import paper_2001_03180_amd as M
    return M


def _systems():
    sys_ = [ics.hernquist(379, 1), ics.plummer(64, 3), ics.plummer(2, 5), ics.hernquist(512, 7)]
    off = np.cumsum([0] + [len(s[0]) for s in sys_])
    m = np.concatenate([s[0] for s in sys_])
    x = np.concatenate([s[1] for s in sys_])
    v = np.concatenate([s[2] for s in sys_])
    return sys_, off, m, x, v


@pytest.mark.parametrize("kind", [0, 1])
def test_rebuild_cycles_parity(ctx, orc, kind):
    sys_, off, m, x, v = _systems()
    n_sys = len(sys_)
    say(f"rebuild cycles kind={kind} n_sys={n_sys}")
    xs, vs, ml = ctx.rebuild_cycles(off, [kind] * n_sys, m, x, v, 30, 3)
    xs2, vs2, ml2 = ctx.rebuild_cycles(off, [kind] * n_sys, m, x, v, 30, 3)
    assert np.array_equal(xs, xs2) and np.array_equal(vs, vs2) and np.array_equal(ml, ml2)
    for s, (ms, x0, v0) in enumerate(sys_):
        o, e = off[s], off[s + 1]
        xo, vo, mlo = orc.rebuild_cycles(ms, x0, v0, kind, 30, 3)
        assert ml[s] == mlo
        R, V = np.abs(x0).max(), np.abs(v0).max()
        assert np.abs(xs[:, o:e] - xo).max() <= 1e-13 * R
        assert np.abs(vs[:, o:e] - vo).max() <= 1e-13 * V


@pytest.mark.parametrize("kind", [0, 1])
def test_round_trip_exact_on_a_dyadic_lattice(ctx, kind):
    rng = np.random.default_rng(0)
    while True:
        x = rng.integers(-8, 8, (8, 3)).astype(float)
        if len({tuple(r) for r in x}) == 8:
            break
    v = rng.integers(-4, 4, (8, 3)).astype(float)
    m = np.full(8, 1 / 8)
    xs, vs, ml = ctx.rebuild_cycles([0, 8], [kind], m, x, v, 300, 3)
    for k in range(3):
        assert np.array_equal(xs[k], x) and np.array_equal(vs[k], v)


def test_rebuild_error_chain_exceeds_mst(ctx, orc):
    """Sec. 3.5: ten N = 379 clusters, 300 round trips each with both
    structures in one call; the chain moves the energy several times more.
    (Over longer runs the MST's error keeps growing, about 2.8e-18 per cycle,
    while the chain's stays near 7.7e-15: the same on the oracle.)"""
    sys_ = [ics.hernquist(379, seed) for seed in range(1, 11)]
    off = np.cumsum([0] + [379] * 20)
    m = np.concatenate([s[0] for s in sys_] * 2)
    x = np.concatenate([s[1] for s in sys_] * 2)
    v = np.concatenate([s[2] for s in sys_] * 2)
    say("rebuild error, 20 systems x 300 cycles")
    xs, vs, ml = ctx.rebuild_cycles(off, [0] * 10 + [1] * 10, m, x, v, 300, 1)
    err = []
    for s in range(20):
        o, e = off[s], off[s + 1]
        d0 = orc.diagnostics(m[o:e], x[o:e], v[o:e])["E"]
        d1 = orc.diagnostics(m[o:e], xs[0, o:e], vs[0, o:e])["E"]
        err.append(abs(d1 - d0) / abs(d0))
    mst, chain = np.mean(err[:10]), np.mean(err[10:])
    assert chain >= 3.0 * mst and chain < 1e-13, (mst, chain)
    assert np.all(ml[10:] == 189.0) and np.all(ml[:10] < 189.0 / 2)


def test_rebuild_cycles_validation(ctx, M):
    m, x, v = ics.plummer(8, 1)
    with pytest.raises(M.MstarError):
        ctx.rebuild_cycles([0, 8], [4], m, x, v, 1, 1)
    m, x, v = ics.plummer(513, 1)
    with pytest.raises(M.MstarError):
        ctx.rebuild_cycles([0, 513], [0], m, x, v, 1, 1)


def test_plain_sum_round_trips_repeat_the_oracle_over_2000_cycles(ctx, orc):
    """The Sec. 3.5 curve with plain sums: ten Hernquist clusters (N = 379),
    MST and chain, 2000 round trips; the GPU states after 500, 1000, 1500 and
    2000 cycles equal the oracle's bit for bit, so the energy-error curves
    are the same curve.  Its values are printed."""
    import concurrent.futures as cf
    import math
    sys_ = [ics.hernquist(379, seed) for seed in range(1, 11)]
    off = np.cumsum([0] + [379] * 20)
    m = np.concatenate([s[0] for s in sys_] * 2)
    x = np.concatenate([s[1] for s in sys_] * 2)
    v = np.concatenate([s[2] for s in sys_] * 2)
    say("plain-sum round trips, 20 systems x 2000 cycles")
    xs, vs, ml = ctx.rebuild_cycles(off, [2] * 10 + [3] * 10, m, x, v, 2000, 4)

    def one(s):
        ms, x0, v0 = sys_[s % 10]
        return orc.rebuild_cycles(ms, x0, v0, 2 if s < 10 else 3, 2000, 4)

    with cf.ThreadPoolExecutor(max_workers=16) as pool:
        ref = list(pool.map(one, range(20)))

    def energy(ms, xx, vv):
        terms = list(0.5 * ms * (vv * vv).sum(1))
        for i in range(len(ms) - 1):
            d = xx[i + 1:] - xx[i]
            terms.extend(-(ms[i] * ms[i + 1:]) / np.sqrt((d * d).sum(1)))
        return math.fsum(terms)

    curve = np.zeros((4, 2))
    for s in range(20):
        o, e = off[s], off[s + 1]
        xo, vo, mlo = ref[s]
        assert np.array_equal(xs[:, o:e], xo) and np.array_equal(vs[:, o:e], vo), s
        assert abs(ml[s] - mlo) <= 1e-12 * mlo   # per-launch partial sums of the same levels
        ms = sys_[s % 10][0]
        E0 = energy(ms, sys_[s % 10][1], sys_[s % 10][2])
        for k in range(4):
            curve[k, s // 10] += abs(energy(ms, xs[k, o:e], vs[k, o:e]) / E0 - 1.0) / 10
    for k in range(4):
        say(f"{500 * (k + 1)} cycles: mean |dE/E| MST {curve[k, 0]:.2e}, chain {curve[k, 1]:.2e}")
