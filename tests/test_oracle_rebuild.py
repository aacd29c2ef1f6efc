"""Pins of the oracle's chain builder and coordinate round trips (Sec. 2.2,
Sec. 3.5), the references of the GPU rebuild-cycle kernel."""
import numpy as np
import pytest

import ics


def _path_checks(parent, level, order, n):
    assert sorted(level) == list(range(n))                  # a path: one body per level
    assert order[0] == int(np.argmin(level)) and parent[order[0]] == -1
    for k in range(1, n):
        assert parent[order[k]] == order[k - 1]
        assert level[order[k]] == k


def test_chain_on_a_line_is_the_sorted_order(orc):
    """Points on a line with growing gaps: the shortest edge is (0, 1) and each
    next point is nearest to the growing end, so the chain is the line order."""
    xs = np.array([0.0, 1.0, 3.0, 7.0, 15.0, 31.0])
    perm = np.array([3, 0, 5, 1, 4, 2])
    x = np.zeros((6, 3))
    x[perm, 0] = xs
    parent, level, order = orc.chain(x)
    _path_checks(parent, level, order, 6)
    along = x[order, 0]
    assert np.all(np.diff(along) > 0) or np.all(np.diff(along) < 0)


@pytest.mark.parametrize("n,seed", [(5, 1), (9, 2), (40, 3)])
def test_chain_is_a_path_through_the_shortest_edge(orc, n, seed):
    x = np.random.default_rng(seed).standard_normal((n, 3))
    parent, level, order = orc.chain(x)
    _path_checks(parent, level, order, n)
    d = np.linalg.norm(x[:, None] - x[None], axis=2)
    d[np.arange(n), np.arange(n)] = np.inf
    i, j = np.unravel_index(np.argmin(d), d.shape)
    assert parent[i] == j or parent[j] == i                 # the first edge stays in the chain
    assert level.mean() == (n - 1) / 2                      # Sec. 3.5: <L_chain> = (N - 1)/2


@pytest.mark.parametrize("kind", [0, 1])
def test_round_trip_is_exact_on_a_dyadic_lattice(orc, kind):
    """With integer coordinates and masses 1/8 every sum in the round trip is
    exact: the state must come back bit for bit, cycle after cycle."""
    rng = np.random.default_rng(0)
    while True:
        x = rng.integers(-8, 8, (8, 3)).astype(float)
        if len({tuple(r) for r in x}) == 8:
            break
    v = rng.integers(-4, 4, (8, 3)).astype(float)
    m = np.full(8, 1 / 8)
    xs, vs, ml = orc.rebuild_cycles(m, x, v, kind, 300, 3)
    for k in range(3):
        assert np.array_equal(xs[k], x) and np.array_equal(vs[k], v)


def test_mst_mean_level_is_below_the_chain(orc):
    """Sec. 3.5 (figure of mean levels): rooted near the centre of mass, the MST
    is several times shallower than the chain (the paper's figure: a factor of
    2 to 10 for N = 10 .. 1000; these Hernquist samples give about 3, 10 and
    19 at N = 30, 379, 1000)."""
    for n, seed in [(30, 1), (379, 1), (1000, 2)]:
        m, x, v = ics.hernquist(n, seed)
        _, _, ml_mst = orc.rebuild_cycles(m, x, v, 0, 1, 0)
        _, _, ml_chain = orc.rebuild_cycles(m, x, v, 1, 1, 0)
        assert ml_chain == (n - 1) / 2
        assert ml_chain / ml_mst >= 2.0, (n, ml_chain / ml_mst)


def test_rebuild_error_chain_exceeds_mst(orc):
    """Sec. 3.5 (rebuild test): repeated build/deconstruct round trips of an
    N = 379 cluster move the energy about an order of magnitude more with the
    chain than with the MST (mean over seeds)."""
    err = {0: [], 1: []}
    for seed in range(1, 6):
        m, x, v = ics.hernquist(379, seed)
        E0 = orc.diagnostics(m, x, v)["E"]
        for kind in (0, 1):
            xs, vs, _ = orc.rebuild_cycles(m, x, v, kind, 300, 1)
            err[kind].append(abs(orc.diagnostics(m, xs[0], vs[0])["E"] - E0) / abs(E0))
    ratio = np.mean(err[1]) / np.mean(err[0])
    assert ratio >= 3.0, ratio
    assert np.mean(err[1]) < 1e-13
