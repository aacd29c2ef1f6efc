"""Pin of the oracle's new-edge rule at an MST rebuild (Sec. 3.5).

Reading: each edge vector of the new tree is the separation the old tree gives
for that pair under the close-pair rule (eq. LCA).  Its defining consequence:
an edge both trees share keeps the exact bits of its position and velocity
vectors, and an edge the new tree only reverses is negated exactly, so a
rebuild adds no rounding to the pairs the old tree already held.  The plain
reading X_v = rho_v - rho_parent (differences of the deconstructed positions)
breaks both, which is what this pin detects.
"""
import numpy as np

import ics


def _moved_state(orc, n, seed, dt):
    """A state whose tree is the MST of the start positions while the bodies
    have moved on by dt v: the old tree's edge vectors of the moved bodies."""
    m, x, v = ics.plummer(n, seed)
    parent, X, V, scal = orc.build_state(m, x, v)
    x2 = x + dt * v
    X2 = np.zeros_like(X)
    for u in range(n):
        if parent[u] >= 0:
            X2[u] = x2[u] - x2[parent[u]]
    return m, parent, X2, V, scal


def test_rebuild_keeps_persisting_edges_bit_for_bit(orc):
    m, parent, X, V, scal = _moved_state(orc, 300, 4, 0.08)
    n = len(m)
    for nd in (1, 2, 4):
        newp, nX, nV, changed = orc.rebuild_state(m, parent, X, V, scal, orc.params(n_d=nd))
        assert changed
        kept = [u for u in range(n) if newp[u] >= 0 and newp[u] == parent[u]]
        rev = [u for u in range(n) if newp[u] >= 0 and parent[newp[u]] == u]
        assert len(kept) > n // 2 and len(kept) < n - 1 and len(rev) > 0
        for u in kept:
            assert np.array_equal(nX[u], X[u]) and np.array_equal(nV[u], V[u]), (nd, u)
        for u in rev:
            q = newp[u]
            assert np.array_equal(nX[u], -X[q]) and np.array_equal(nV[u], -V[q]), (nd, u)
        # the rebuilt tree describes the same bodies
        rho_old = orc.deconstruct(parent, X)
        rho_new = orc.deconstruct(newp, nX)
        root = int(np.nonzero(newp < 0)[0][0])
        d_old = rho_old - rho_old[root]
        scale = np.abs(d_old).max()
        assert np.abs(rho_new - d_old).max() <= 1e-12 * scale


def test_rho_difference_rule_would_change_persisting_bits(orc):
    """The pin above is not vacuous: differences of deconstructed positions
    change the bits of most persisting edges of this state."""
    m, parent, X, V, scal = _moved_state(orc, 300, 4, 0.08)
    rho = orc.deconstruct(parent, X)
    changed = sum(not np.array_equal(rho[u] - rho[parent[u]], X[u]) for u in range(len(m)) if parent[u] >= 0)
    assert changed > len(m) // 4
