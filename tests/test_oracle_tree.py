"""Oracle pins for MST coordinates: deconstruction, the LCA closeness rule
(eq. LCA) and separations (Sec. 3.4)."""
from collections import deque

import numpy as np
import pytest


def random_tree(n, rng, branchy=True):
    parent = np.full(n, -1, dtype=np.int32)
    perm = rng.permutation(n)
    for k in range(1, n):
        j = rng.integers(0, k) if branchy else k - 1
        parent[perm[k]] = perm[j]
    return parent


def bfs_dist(parent, src):
    n = len(parent)
    adj = [[] for _ in range(n)]
    for v, p in enumerate(parent):
        if p >= 0:
            adj[v].append(int(p)); adj[int(p)].append(v)
    dist = [-1] * n
    dist[src] = 0
    q = deque([src])
    while q:
        u = q.popleft()
        for w in adj[u]:
            if dist[w] < 0:
                dist[w] = dist[u] + 1; q.append(w)
    return dist


def path_vertices(parent, v):
    out = []
    while v >= 0:
        out.append(int(v)); v = parent[v]
    return out[::-1]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lca_rule_equals_tree_distance(orc, seed):
    rng = np.random.default_rng(seed)
    n = 40
    parent = random_tree(n, rng, branchy=seed != 2)
    X = rng.standard_normal((n, 3)); X[parent < 0] = 0
    rho = orc.deconstruct(parent, X)
    for nd in range(0, 5):
        for i in range(n):
            dist = bfs_dist(parent, i)
            for j in range(n):
                if i == j:
                    continue
                _, close = orc.separation(i, j, parent, X, rho, nd)
                assert close == (dist[j] <= nd), (nd, i, j, dist[j])


def test_deconstruct_is_root_path_sum(orc):
    rng = np.random.default_rng(5)
    n = 50
    parent = random_tree(n, rng)
    X = rng.standard_normal((n, 3)); X[parent < 0] = 0
    rho = orc.deconstruct(parent, X)
    for v in range(n):
        acc = np.zeros(3)
        for u in path_vertices(parent, v)[1:]:
            acc = acc + X[u]
        assert np.array_equal(acc, rho[v])          # same order: bit-identical


def test_separations_antisymmetric_and_consistent(orc):
    rng = np.random.default_rng(6)
    n = 60
    parent = random_tree(n, rng)
    X = rng.standard_normal((n, 3)); X[parent < 0] = 0
    rho = orc.deconstruct(parent, X)
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            dij, cij = orc.separation(i, j, parent, X, rho, 2)
            dji, cji = orc.separation(j, i, parent, X, rho, 2)
            assert cij == cji
            assert np.array_equal(dij, -dji)
            scale = np.abs(rho).max() + np.abs(X).max()
            assert np.abs(dij - (rho[j] - rho[i])).max() <= 64 * np.finfo(float).eps * scale


def test_close_pair_cases_explicit(orc):
    """The five N_d = 2 cases: child, parent, grandchild, grandparent, sibling."""
    parent = np.array([-1, 0, 1, 1, 2], dtype=np.int32)   # 0 -> 1 -> {2, 3}, 2 -> 4
    X = np.array([[0, 0, 0], [1.0, 0, 0], [0, 2.0, 0], [0, 0, 3.0], [0.5, 0.25, 0.125]])
    rho = orc.deconstruct(parent, X)
    cases = {(1, 2): X[2], (2, 1): -X[2], (1, 4): X[2] + X[4], (4, 1): -(X[4] + X[2]),
             (2, 3): X[3] - X[2], (0, 1): X[1], (0, 2): X[1] + X[2]}
    for (i, j), want in cases.items():
        d, close = orc.separation(i, j, parent, X, rho, 2)
        assert close and np.array_equal(d, want), (i, j)
    d, close = orc.separation(0, 4, parent, X, rho, 2)      # distance 3: Cartesian
    assert not close and np.array_equal(d, rho[4] - rho[0])


def test_mst_path_sum_beats_cartesian_difference(orc):
    """Purpose of MST coordinates (Sec. 2.2, 3.4): a tight pair far from the
    root keeps its separation exactly in the edge vector, while differences of
    root-relative positions lose the low digits."""
    parent = np.array([-1, 0, 1], dtype=np.int32)
    X = np.array([[0, 0, 0], [1e3 + 1 / 3, 2e3, -7e2], [1e-10, -2e-10, 3e-10]])
    rho = orc.deconstruct(parent, X)
    d, close = orc.separation(1, 2, parent, X, rho, 2)
    assert close and np.array_equal(d, X[2])
    cart = rho[2] - rho[1]
    assert np.abs(cart - X[2]).max() / 1e-10 > 1e-8
