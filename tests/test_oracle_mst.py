"""Oracle pins for the minimum spanning tree (paper Sec. 3.1-3.4).

The MST under the strict edge order (w = |d|^2 without FMA, min index, max
index) is unique (Sec. 3.1).  Pins: brute force over all labelled trees
(Pruefer sequences) for N <= 8, an independent Kruskal, the cycle/cut
certificate (Sec. 3.1) on larger sets, integer lattices with massive weight
ties, and the mean-level property of Sec. 3.5.
"""
import itertools

import numpy as np
import pytest


def key(x, i, j):
    d = x[j] - x[i]
    w = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    return (w, min(i, j), max(i, j))


def edges_of(parent):
    return sorted((min(v, int(p)), max(v, int(p))) for v, p in enumerate(parent) if p >= 0)


def pruefer_to_edges(seq, n):
    degree = [1] * n
    for s in seq:
        degree[s] += 1
    edges = []
    for s in seq:
        leaf = min(i for i in range(n) if degree[i] == 1)
        edges.append((min(leaf, s), max(leaf, s)))
        degree[leaf] -= 1
        degree[s] -= 1
    u, w = [i for i in range(n) if degree[i] == 1]
    edges.append((u, w))
    return edges


def brute_force_mst(x):
    n = len(x)
    best = None
    for seq in itertools.product(range(n), repeat=n - 2):
        e = pruefer_to_edges(seq, n)
        keys = sorted(key(x, i, j) for i, j in e)
        if best is None or keys < best[0]:
            best = (keys, sorted(e))
    return best[1]


def kruskal(x):
    n = len(x)
    allk = sorted(key(x, i, j) for i in range(n) for j in range(i + 1, n))
    comp = list(range(n))

    def find(a):
        while comp[a] != a:
            comp[a] = comp[comp[a]]
            a = comp[a]
        return a

    out = []
    for w, i, j in allk:
        a, b = find(i), find(j)
        if a != b:
            comp[a] = b
            out.append((i, j))
    return sorted(out)


@pytest.mark.parametrize("n,seed", [(3, 1), (4, 2), (5, 3), (6, 4), (7, 5), (7, 6)])
def test_prim_matches_brute_force(orc, n, seed):
    x = np.random.default_rng(seed).standard_normal((n, 3))
    root = orc.root_nearest_com(np.ones(n), x)
    parent, level, order = orc.mst(x, root)
    assert edges_of(parent) == brute_force_mst(x)


def test_prim_brute_force_lattice_n8(orc):
    """N = 8 (8^6 labelled trees) on a 2x2x2 cube: all 12 cube edges tie."""
    x = np.array(list(itertools.product(range(2), range(2), range(2))), dtype=float)
    parent, _, _ = orc.mst(x, 5)
    assert edges_of(parent) == brute_force_mst(x)


@pytest.mark.parametrize("shape", [(2, 2, 1), (3, 2, 1), (1, 1, 7)])
def test_lattice_ties_brute_force(orc, shape):
    """Integer lattices: many equal weights; the index tie-break decides.  The
    edge set must not depend on the root."""
    x = np.array(list(itertools.product(*[range(s) for s in shape])), dtype=float)
    want = brute_force_mst(x)
    for root in range(len(x)):
        parent, _, _ = orc.mst(x, root)
        assert edges_of(parent) == want


@pytest.mark.parametrize("n,seed", [(50, 10), (200, 11), (300, 12)])
def test_prim_matches_kruskal(orc, n, seed):
    x = np.random.default_rng(seed).standard_normal((n, 3)) ** 3
    parent, _, _ = orc.mst(x, n // 2)
    assert edges_of(parent) == kruskal(x)


def test_lattice_matches_kruskal(orc):
    x = np.array(list(itertools.product(range(5), range(4), range(3))), dtype=float)
    parent, _, _ = orc.mst(x, 7)
    assert edges_of(parent) == kruskal(x)


def _tree_path(parent, level, i, j):
    a, b = i, j
    pa, pb = [], []
    while level[a] > level[b]:
        pa.append(a); a = parent[a]
    while level[b] > level[a]:
        pb.append(b); b = parent[b]
    while a != b:
        pa.append(a); pb.append(b); a = parent[a]; b = parent[b]
    return [(v, parent[v]) for v in pa + pb]


def test_certificate_cycle_and_cut(orc):
    """Cycle property: every non-tree edge is heavier than every edge on the tree
    path it closes.  Cut property: every tree edge is the lightest edge across
    the cut it defines (Sec. 3.1)."""
    rng = np.random.default_rng(21)
    n = 40
    x = rng.standard_normal((n, 3))
    parent, level, order = orc.mst(x, 3)
    assert sum(parent < 0) == 1 and len(edges_of(parent)) == n - 1
    tree = set(edges_of(parent))
    for i in range(n):
        for j in range(i + 1, n):
            if (i, j) in tree:
                continue
            kij = key(x, i, j)
            for u, w in _tree_path(parent, level, i, j):
                assert key(x, u, w) < kij
    children = {v: [] for v in range(n)}
    for v in range(n):
        if parent[v] >= 0:
            children[int(parent[v])].append(v)
    for v in range(n):
        if parent[v] < 0:
            continue
        sub, stack = set(), [v]
        while stack:
            u = stack.pop(); sub.add(u); stack.extend(children[u])
        kv = key(x, v, int(parent[v]))
        for a in sub:
            for b in range(n):
                if b not in sub and (min(a, b), max(a, b)) != (min(v, parent[v]), max(v, parent[v])):
                    assert kv < key(x, a, b)


def test_prim_levels_parents_and_order(orc):
    x = np.random.default_rng(4).standard_normal((40, 3))
    parent, level, order = orc.mst(x, 11)
    assert order[0] == 11 and parent[11] == -1 and level[11] == 0
    pos = {int(v): k for k, v in enumerate(order)}
    for v in range(40):
        if v != 11:
            assert level[v] == level[parent[v]] + 1
            assert pos[int(parent[v])] < pos[v]           # parents are added first
    root2, level2, _ = orc.tree_levels(parent)
    assert root2 == 11 and np.array_equal(level, level2)


def test_root_nearest_com(orc):
    rng = np.random.default_rng(8)
    m = rng.uniform(0.5, 2.0, 100)
    x = rng.standard_normal((100, 3))
    c = np.array([sum(m[i] * x[i, k] for i in range(100)) for k in range(3)]) / m.sum()
    d = x - c
    w = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    assert orc.root_nearest_com(m, x) == int(np.argmin(w))


def test_mean_level_below_chain(orc):
    """Sec. 3.5: rooted near the COM the MST is much shallower than a chain,
    <L_MST> < (N-1)/2 = <L_chain> (paper: ratio ~2-10 for N = 10-1000)."""
    import ics
    for n, seed in [(10, 1), (100, 2), (1000, 3)]:
        m, x, _ = ics.plummer(n, seed)
        parent, level, _ = orc.mst(x, orc.root_nearest_com(m, x))
        ratio = ((n - 1) / 2) / level.mean()
        assert ratio > 1.5
