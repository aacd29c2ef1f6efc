"""GPU divide-and-conquer spanning tree (Sec. 3.3) against the oracle's, through the C ABI.

The groups, each group's minimum spanning tree and the meta-graph's are all
defined exactly (strict edge order, the octree reading), so the GPU tree must
equal the oracle's bit for bit: parent, level and root.  The integrators with
MSTAR_MST_DC follow the oracle's driver with mst_method = 1 (replay mode, and free
mode up to a flipped step decision).
"""
import sys

import numpy as np
import pytest

import ics

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-dc] {msg}", flush=True)
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


def _lattice():
    return np.array([[i, j, k] for i in range(6) for j in range(6) for k in range(6)], float)


CASES = {
    "two": lambda: (np.array([0.3, 0.7]), np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 3.0]])),
    "plummer64": lambda: ics.plummer(64, 5)[:2],
    "plummer300": lambda: ics.plummer(300, 7)[:2],
    "binary600": lambda: ics.plummer_with_binary(598, 11)[:2],
    "uniform1025": lambda: (np.full(1025, 1.0 / 1025), np.random.default_rng(3).uniform(-1, 1, (1025, 3))),
    "lattice216": lambda: (np.full(216, 1.0 / 216), _lattice()),
    "collinear100": lambda: (np.full(100, 0.01), np.stack([np.linspace(0, 1, 100) ** 2, np.zeros(100), np.zeros(100)], 1)),
    "plummer1000_bh": lambda: ics.workload("plummer1000_bh")[:2],
    "plummer5000_binary": lambda: ics.workload("plummer5000_binary")[:2],
    "plummer10000_binary": lambda: ics.workload("plummer10000_binary")[:2],
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_dc_tree_parity(ctx, orc, name):
    m, x = CASES[name]()
    say(f"{name}: N={len(m)}")
    parent, level, root = ctx.mst_build(m, x, dc=True)
    r = orc.root_nearest_com(m, x)
    po, lo, oo, part, npart = orc.mst_dc(x, r)
    assert root == r
    assert np.array_equal(parent, po), (name, int(np.sum(parent != po)))
    assert np.array_equal(level, lo)
    say(f"{name}: {npart} groups, identical")


def test_dc_device_pointers(ctx, orc):
    import torch
    m, x = ics.plummer(300, 7)[:2]
    p_dev, l_dev, root = ctx.mst_build(torch.tensor(m, device="cuda"), torch.tensor(x, device="cuda"), dc=True)
    po = orc.mst_dc(x, orc.root_nearest_com(m, x))[0]
    assert np.array_equal(p_dev.cpu().numpy(), po)


def test_dc_exact_flag_still_exact(ctx, orc):
    """The exact builder is unchanged next to the divide-and-conquer one."""
    m, x = ics.plummer(300, 7)[:2]
    r = orc.root_nearest_com(m, x)
    parent, level, root = ctx.mst_build(m, x)
    assert np.array_equal(parent, orc.mst(x, r)[0])
    parent2, _, _ = ctx.mst_build(m, x, dc=True)
    assert not np.array_equal(parent, parent2)


def _rel(xg, vg, xo, vo, m):
    rcm = (m[:, None] * xo).sum(0) / m.sum()
    vcm = (m[:, None] * vo).sum(0) / m.sum()
    return np.abs(xg - xo).max() / np.abs(xo - rcm).max(), np.abs(vg - vo).max() / np.abs(vo - vcm).max()


@pytest.mark.parametrize("name,t_end", [("plummer64", 0.5), ("plummer1000_bh", 0.02)])
def test_dc_integration_parity(ctx, orc, M, name, t_end):
    """The integrator with divide-and-conquer trees (initial build and every
    rebuild) against the oracle's driver with mst_method = 1.

    Replay mode: the oracle repeats the GPU's recorded accepted steps with its
    own divide-and-conquer builds and rebuilds; end states agree to 1e-11 of
    the system's extent and velocity spread.  Free mode: the step counts may
    differ by a flipped accept/reject decision (an error measure within
    rounding of eta), the end states agree to 1e-10 and the energy errors to
    1e-13."""
    if name == "plummer64":
        m, x, v = ics.plummer(64, 5)
    else:
        m, x, v, wl = ics.workload(name)
    say(f"integrate {name} to t={t_end} with divide-and-conquer trees")
    p = M.params(eta=1e-12)
    p.flags |= M.MST_DC
    po = orc.params(eta=1e-12, mst_method=1)
    xg, vg, rc, st, H = ctx.integrate_record(m, x, v, 0.0, t_end, 100000, p)
    assert rc == 0 and len(H) == st["steps_accepted"]
    xr, vr, tr = orc.replay(m, x, v, 0.0, H, None, po)
    ex, ev = _rel(xg, vg, xr, vr, m)
    say(f"{name}: replay of {len(H)} steps: state {ex:.1e} {ev:.1e}")
    assert ex <= 1e-11 and ev <= 1e-11
    xo, vo, rco, sto = orc.integrate(m, x, v, 0.0, t_end, po)
    assert rco == 0
    say(f"{name}: steps gpu {st['steps_accepted']}+{st['steps_rejected']} oracle "
        f"{sto['steps_accepted']}+{sto['steps_rejected']}, rebuilds {st['mst_rebuilds']}")
    assert abs(st["steps_accepted"] - sto["steps_accepted"]) <= 1
    assert abs(st["steps_rejected"] - sto["steps_rejected"]) <= 2
    ex, ev = _rel(xg, vg, xo, vo, m)
    E0 = orc.diagnostics(m, x, v)["E"]
    dg = orc.diagnostics(m, xg, vg)["E"] / E0 - 1.0
    do = orc.diagnostics(m, xo, vo)["E"] / E0 - 1.0
    say(f"{name}: free mode state {ex:.1e} {ev:.1e}; dE/E gpu {dg:.1e} oracle {do:.1e}")
    assert ex <= 1e-10 and ev <= 1e-10
    assert abs(dg - do) <= 1e-13
