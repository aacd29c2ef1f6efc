"""GPU (HIP, gfx950) path vs the CPU oracle, stage by stage, through the C ABI.

Tolerances (derived from the arithmetic of each stage):
  * MST edge set: bit-exact (same positions, same no-FMA weights, same
    strict edge order); parent/level identical when the roots agree.
  * one force evaluation: max_i |a_i - a_i^oracle| / (G sum_j m_j/r_ij^2)
    <= 1e-13 and |dU/U| <= 1e-13 (summation order and 1/sqrt rounding).
  * leapfrog / GBS step end states: relative to the state scale, 1e-12.
  * free integrations inside the predictability horizon: 1e-10 (positions
    relative to max|r - r_cm|, velocities relative to max|v - v_cm|).
Every GPU result is computed twice and must be bitwise identical.
"""
import math
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


def edges(parent):
    return sorted((min(v, int(p)), max(v, int(p))) for v, p in enumerate(parent) if p >= 0)


def lattice(k):
    g = np.arange(k, dtype=float)
    return np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T.copy()


MST_CASES = [
    ("random8", lambda: (np.ones(8), np.random.default_rng(1).standard_normal((8, 3)))),
    ("lattice4", lambda: (np.ones(64), lattice(4))),
    ("lattice5_ragged", lambda: (np.ones(125), lattice(5))),
    ("plummer1001", lambda: ics.plummer_with_central_mass(1000, 201)[:2]),
    ("plummer5002_binary", lambda: ics.plummer_with_binary(5000, 301)[:2]),
]


@pytest.mark.parametrize("name,make", MST_CASES, ids=[c[0] for c in MST_CASES])
def test_mst_parity(ctx, orc, name, make):
    m, x = make()
    say(f"mst_build {name} n={len(m)}")
    parent, level, root = ctx.mst_build(m, x)
    parent2, level2, root2 = ctx.mst_build(m, x)
    assert np.array_equal(parent, parent2) and np.array_equal(level, level2) and root == root2
    ro = orc.root_nearest_com(m, x)
    po, lo, _ = orc.mst(x, ro)
    assert edges(parent) == edges(po)
    if root == ro:
        assert np.array_equal(parent, po) and np.array_equal(level, lo)
    # rooted at the oracle's root, parents and levels must match exactly
    parent3, level3, root3 = ctx.mst_build(m, x, root_in=ro)
    assert root3 == ro and np.array_equal(parent3, po) and np.array_equal(level3, lo)


def _edge_rel_ok(Xg, Xo, tol=1e-12):
    """Every MST edge against its own length (a hard binary's edge is ~1e-4 of
    the cluster's size), with a floor of 1e-16 of the longest edge for rows
    at the rounding level (the root row is zero)."""
    lo = np.linalg.norm(Xo, axis=1)
    d = np.linalg.norm(Xg - Xo, axis=1)
    bad = d > tol * lo + 1e-16 * lo.max()
    return not bad.any(), float((d / np.maximum(lo, 1e-300))[lo > 0].max())


def _state(orc, m, x, v):
    parent, X, V, scal = orc.build_state(m, x, v)
    rho = orc.deconstruct(parent, X)
    _, _, U, _, _ = orc.force(m, parent, X, rho)
    vt = v - (m[:, None] * v).sum(0) / m.sum()
    scal[1] = U - 0.5 * (m * (vt ** 2).sum(1)).sum()
    return parent, X, V, scal, rho


FORCE_CASES = [("plummer32", 32, 101), ("plummer200_ragged", 200, 7), ("plummer1001", 1001, 201),
               ("binary5002", 5002, 301), ("binary10002", 10002, 302)]


def _scale(m, rho):
    n = len(m)
    s = np.empty(n)
    for i in range(n):
        d = rho - rho[i]
        r2 = (d * d).sum(1)
        r2[i] = np.inf
        s[i] = (m / r2).sum()
    return s


@pytest.mark.parametrize("name,n,seed", FORCE_CASES, ids=[c[0] for c in FORCE_CASES])
@pytest.mark.parametrize("nd", [0, 1, 2, 3, 4])
def test_force_parity(ctx, orc, M, name, n, seed, nd):
    if n in (5002, 10002):
        m, x, v = ics.plummer_with_binary(n - 2, seed)
    elif n == 1001:
        m, x, v = ics.plummer_with_central_mass(1000, seed)
    else:
        m, x, v = ics.plummer(n, seed)
    parent, X, V, scal, rho = _state(orc, m, x, v)
    say(f"force {name} n={n} nd={nd}")
    p = M.params(n_d=nd)
    acc, U = ctx.force(m, rho, parent, X, p)
    acc2, U2 = ctx.force(m, rho, parent, X, p)
    assert np.array_equal(acc, acc2) and U == U2
    ao, _, Uo, _, _ = orc.force(m, parent, X, rho, orc.params(n_d=nd, nthreads=0))
    err = np.abs(acc - ao).max(1) / _scale(m, rho)
    assert err.max() <= 1e-13, err.max()
    assert abs(U - Uo) <= 1e-13 * Uo


@pytest.fixture(scope="module")
def ctx_kinds():
    """One context per force kernel (MSTAR_FORCE_KERNEL is read when a context
    is created): the pairwise kernel, and the mutual (i < j) kernel at any N."""
    import os
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_03180_amd as M
    old = os.environ.get("MSTAR_FORCE_KERNEL")
    out = {}
    try:
        for kind in ("pairwise", "mutual"):
            os.environ["MSTAR_FORCE_KERNEL"] = kind
            out[kind] = M.Context(0)
    finally:
        if old is None:
            os.environ.pop("MSTAR_FORCE_KERNEL", None)
        else:
            os.environ["MSTAR_FORCE_KERNEL"] = old
    yield out
    for c in out.values():
        c.close()


KIND_CASES = [("plummer32", 32, 101), ("plummer65_ragged", 65, 3), ("plummer200_ragged", 200, 7),
              ("plummer1001", 1001, 201), ("binary5002", 5002, 301), ("binary20002_ragged", 20002, 303)]


_KIND_STATE = {}


@pytest.mark.parametrize("name,n,seed", KIND_CASES, ids=[c[0] for c in KIND_CASES])
@pytest.mark.parametrize("nd", [0, 2])
@pytest.mark.parametrize("kind", ["pairwise", "mutual"])
def test_force_parity_kernels(ctx_kinds, orc, M, kind, name, n, seed, nd):
    """Both force kernels against the oracle at sizes with full and ragged
    64-body blocks (the mutual kernel's rows of 256 bodies, its diagonal
    blocks and padding), each result bitwise reproducible."""
    if n in (5002, 20002):   # 20002: past the largest N the mutual kernel takes by default, ragged rows
        m, x, v = ics.plummer_with_binary(n - 2, seed)
    elif n == 1001:
        m, x, v = ics.plummer_with_central_mass(1000, seed)
    else:
        m, x, v = ics.plummer(n, seed)
    if name not in _KIND_STATE:   # the state and its force scale serve every kernel and N_d
        parent, X, V, scal, rho = _state(orc, m, x, v)
        _KIND_STATE[name] = (parent, X, rho, _scale(m, rho))
    parent, X, rho, sc = _KIND_STATE[name]
    say(f"force kernel={kind} {name} n={n} nd={nd}")
    c = ctx_kinds[kind]
    p = M.params(n_d=nd)
    acc, U = c.force(m, rho, parent, X, p)
    acc2, U2 = c.force(m, rho, parent, X, p)
    assert np.array_equal(acc, acc2) and U == U2
    ao, _, Uo, _, _ = orc.force(m, parent, X, rho, orc.params(n_d=nd, nthreads=0))
    err = np.abs(acc - ao).max(1) / sc
    assert err.max() <= 1e-13, err.max()
    assert abs(U - Uo) <= 1e-13 * Uo


@pytest.mark.parametrize("kind", ["pairwise", "mutual"])
def test_gbs_step_parity_kernels(ctx_kinds, orc, M, kind):
    """A GBS step (72 + 1 force evaluations, lane-packed launches of 1..5
    evaluations, each split over waves differently) with either kernel."""
    m, x, v = ics.plummer(300, 17)
    parent, X, V, scal, _ = _state(orc, m, x, v)
    say(f"gbs_step kernel={kind} n=300")
    p = M.params(k_fix=8, eta=1e-12)
    Xg, Vg, sg, acc, eps, hn = ctx_kinds[kind].gbs_step(m, parent, X, V, scal, 0.002, p)
    Xo, Vo, so, acco, epso, hno, nf = orc.gbs_step(m, parent, X, V, scal, 0.002, orc.params(k_fix=8, eta=1e-12))
    eps_tol = 1e-3 * epso + 5e-13
    assert abs(eps - epso) <= eps_tol, (eps, epso)
    assert acc == acco == 1
    assert np.abs(Xg - Xo).max() <= 1e-12 * np.abs(Xo).max()
    assert np.abs(Vg - Vo).max() <= 1e-12 * np.abs(Vo).max()


def test_force_close_pairs_matter(ctx, orc, M):
    """A tight pair far from the origin: the MST path sum keeps digits that the
    Cartesian difference loses; GPU and oracle both use the path sum."""
    m = np.array([1.0, 1e-3, 1e-3, 0.5])
    x = np.array([[0.0, 0.0, 0.0], [1e3, 2e3, -7e2], [1e3 + 1e-9, 2e3 - 2e-9, -7e2 + 3e-9], [5.0, 1.0, 2.0]])
    parent = np.array([-1, 0, 1, 0], dtype=np.int32)
    X = np.array([[0, 0, 0], x[1] - x[0], [1e-9, -2e-9, 3e-9], x[3] - x[0]])
    rho = orc.deconstruct(parent, X)
    acc, U = ctx.force(m, rho, parent, X, M.params(n_d=2))
    ao, _, Uo, _, _ = orc.force(m, parent, X, rho)
    np.testing.assert_allclose(acc, ao, rtol=1e-13, atol=0)
    assert abs(U - Uo) <= 1e-13 * Uo


LF_CASES = [(32, 101, 0.02, 1), (32, 101, 0.05, 5), (200, 7, 0.01, 3), (1001, 201, 0.002, 2)]


@pytest.mark.parametrize("n,seed,H,nsub", LF_CASES)
def test_leapfrog_parity(ctx, orc, M, n, seed, H, nsub):
    if n == 1001:
        m, x, v = ics.plummer_with_central_mass(1000, seed)
    else:
        m, x, v = ics.plummer(n, seed)
    parent, X, V, scal, _ = _state(orc, m, x, v)
    say(f"leapfrog n={n} H={H} nsub={nsub}")
    Xg, Vg, sg = ctx.leapfrog(m, parent, X, V, scal, H, nsub)
    Xg2, Vg2, sg2 = ctx.leapfrog(m, parent, X, V, scal, H, nsub)
    assert np.array_equal(Xg, Xg2) and np.array_equal(Vg, Vg2) and np.array_equal(sg, sg2)
    Xo, Vo, so, nf = orc.leapfrog(m, parent, X, V, scal, H, nsub)
    assert np.abs(Xg - Xo).max() <= 1e-12 * np.abs(Xo).max()
    assert np.abs(Vg - Vo).max() <= 1e-12 * np.abs(Vo).max()
    for a, b in ((Xg, Xo), (Vg, Vo)):
        ok, worst = _edge_rel_ok(a, b)
        assert ok, worst
    assert abs(sg[0] - so[0]) <= 1e-13 * abs(so[0])
    np.testing.assert_allclose(sg[3:6], so[3:6], atol=1e-15)


@pytest.mark.parametrize("n,seed,H,kf", [(32, 101, 0.05, 8), (32, 102, 0.5, 8), (200, 9, 0.01, 4),
                                         (1001, 201, 0.005, 8)])
def test_gbs_step_parity(ctx, orc, M, n, seed, H, kf):
    if n == 1001:
        m, x, v = ics.plummer_with_central_mass(1000, seed)
    else:
        m, x, v = ics.plummer(n, seed)
    parent, X, V, scal, _ = _state(orc, m, x, v)
    say(f"gbs_step n={n} H={H} k_fix={kf}")
    p = M.params(k_fix=kf, eta=1e-12)
    Xg, Vg, sg, acc, eps, hn = ctx.gbs_step(m, parent, X, V, scal, H, p)
    out2 = ctx.gbs_step(m, parent, X, V, scal, H, p)
    assert np.array_equal(Xg, out2[0]) and np.array_equal(Vg, out2[1]) and eps == out2[4]
    Xo, Vo, so, acco, epso, hno, nf = orc.gbs_step(m, parent, X, V, scal, H, orc.params(k_fix=kf, eta=1e-12))
    # eps is a difference of two extrapolations; division end states that agree
    # to ~1e-15 relative enter it through Neville weights of total size ~2e2, so
    # the two error measures may differ by ~2e2 * 1e-15 (x a safety factor 2.5).
    eps_tol = 1e-3 * epso + 5e-13
    assert abs(eps - epso) <= eps_tol, (eps, epso)
    if abs(epso - 1e-12) > eps_tol:
        assert acc == acco
    if acc and acco:
        assert np.abs(Xg - Xo).max() <= 1e-12 * np.abs(Xo).max()
        assert np.abs(Vg - Vo).max() <= 1e-12 * np.abs(Vo).max()
        for a, b in ((Xg, Xo), (Vg, Vo)):
            ok, worst = _edge_rel_ok(a, b)
            assert ok, worst
        assert abs(sg[0] - so[0]) <= 1e-14 * abs(so[0]) + 1e-16
        # h_next ~ eps^(-1/(2k-1)): relative spread <= |d eps / eps| / (2k - 1)
        assert abs(hn - hno) <= (eps_tol / epso / (2 * kf - 1) + 1e-14) * hno
    elif not acc:
        assert np.array_equal(Xg, X) and hn == 0.5 * H


@pytest.mark.parametrize("n_stars,seed", [(5000, 301), (10000, 302)])
def test_gbs_step_parity_full_size(ctx, orc, M, n_stars, seed):
    """One GBS step of the benchmark workload (N_p = 5002, k_fix = 8, eta = 1e-13)
    in the launch configuration the benchmark times, and of its larger size
    (N_p = 10002), against the oracle."""
    m, x, v = ics.plummer_with_binary(n_stars, seed)
    parent, X, V, scal, _ = _state(orc, m, x, v)
    H = 5e-5
    say(f"gbs_step n={len(m)} H={H} k_fix=8")
    p = M.params(k_fix=8, eta=1e-13)
    Xg, Vg, sg, acc, eps, hn = ctx.gbs_step(m, parent, X, V, scal, H, p)
    Xo, Vo, so, acco, epso, hno, nf = orc.gbs_step(m, parent, X, V, scal, H,
                                                   orc.params(k_fix=8, eta=1e-13, nthreads=0))
    assert nf == 8 * 9 + 1
    eps_tol = 1e-3 * epso + 5e-13
    assert abs(eps - epso) <= eps_tol, (eps, epso)
    assert acc == acco == 1
    assert np.abs(Xg - Xo).max() <= 1e-12 * np.abs(Xo).max()
    assert np.abs(Vg - Vo).max() <= 1e-12 * np.abs(Vo).max()
    assert abs(sg[0] - so[0]) <= 1e-14 * abs(so[0]) + 1e-16
    # every edge against its own length, the binary's (the last two bodies) shown
    b = len(m) - 1
    for a, o, what in ((Xg, Xo, "X"), (Vg, Vo, "V")):
        ok, worst = _edge_rel_ok(a, o)
        rb = np.linalg.norm(a[b] - o[b]) / np.linalg.norm(o[b]) if parent[b] >= 0 else 0.0
        say(f"  per-edge worst relative {what}: {worst:.2e}; binary edge {rb:.2e}")
        assert ok, worst


def _rel_state_err(xg, vg, xo, vo, m):
    rc = (m[:, None] * xo).sum(0) / m.sum()
    vc = (m[:, None] * vo).sum(0) / m.sum()
    R = np.abs(xo - rc).max()
    Vs = np.abs(vo - vc).max()
    return np.abs(xg - xo).max() / R, np.abs(vg - vo).max() / Vs


@pytest.mark.parametrize("name,t_end,nd", [("plummer32", 0.1, 2), ("plummer32", 0.3, 2), ("plummer32", 0.1, 4),
                                           ("plummer32", 0.1, 3)])
def test_integrate_parity_plummer32(ctx, orc, M, name, t_end, nd):
    m, x, v, _ = ics.workload(name)
    say(f"integrate {name} t_end={t_end} n_d={nd}")
    xg, vg, rc, st = ctx.integrate(m, x, v, 0.0, t_end, M.params(eta=1e-12, n_d=nd))
    xg2, vg2, _, st2 = ctx.integrate(m, x, v, 0.0, t_end, M.params(eta=1e-12, n_d=nd))
    assert np.array_equal(xg, xg2) and np.array_equal(vg, vg2)
    xo, vo, rco, sto = orc.integrate(m, x, v, 0.0, t_end, orc.params(eta=1e-12, n_d=nd))
    assert rc == rco == 0
    assert abs(st["t_reached"] - sto["t_reached"]) <= 2e-14 * t_end
    ex, ev = _rel_state_err(xg, vg, xo, vo, m)
    assert ex <= 1e-10 and ev <= 1e-10, (ex, ev)
    d0 = orc.diagnostics(m, x, v)
    dg = orc.diagnostics(m, xg, vg)
    do = orc.diagnostics(m, xo, vo)
    dEg = (dg["E"] - d0["E"]) / d0["E"]
    dEo = (do["E"] - d0["E"]) / d0["E"]
    assert abs(dEg) <= 1e-13 and abs(dEg - dEo) <= 1e-13


def test_integrate_kepler_closed_form(ctx, M):
    from tests import kepler
    m, x, v = ics.kepler_two_body(0.5, 0.5, 1.0, 0.9, seed=3)
    tend = 3.3 * 2 * math.pi
    say("integrate kepler e=0.9")
    xg, vg, rc, st = ctx.integrate(m, x, v, 0.0, tend, M.params(eta=1e-12))
    assert rc == 0 and abs(st["t_reached"] - tend) <= 1e-14 * tend
    r, u = kepler.propagate(1.0, x[1] - x[0], v[1] - v[0], st["t_reached"])
    assert np.abs((xg[1] - xg[0]) - r).max() < 5e-12 * np.linalg.norm(r)


def test_integrate_parity_central_mass_short(ctx, orc, M):
    m, x, v, _ = ics.workload("plummer1000_bh")
    say("integrate plummer1000_bh t_end=0.01")
    xg, vg, rc, st = ctx.integrate(m, x, v, 0.0, 0.01, M.params(eta=1e-13))
    xo, vo, rco, sto = orc.integrate(m, x, v, 0.0, 0.01, orc.params(eta=1e-13))
    assert rc == rco == 0
    ex, ev = _rel_state_err(xg, vg, xo, vo, m)
    assert ex <= 1e-10 and ev <= 1e-10, (ex, ev)


def test_error_paths(ctx, M):
    m, x, v = ics.plummer(8, 3)
    say("error paths")
    xb = x.copy(); xb[2] = xb[5]
    with pytest.raises(M.MstarError) as e:
        ctx.integrate(m, xb, v, 0.0, 1.0)
    assert e.value.code == M.E_COINCIDENT
    xb = x.copy(); xb[1, 1] = np.inf
    with pytest.raises(M.MstarError) as e:
        ctx.integrate(m, xb, v, 0.0, 1.0)
    assert e.value.code == M.E_NONFINITE
    with pytest.raises(M.MstarError) as e:
        ctx.integrate(m, x, v, 0.0, 1.0, M.params(n_d=5))
    assert e.value.code == M.E_UNSUPPORTED
    with pytest.raises(M.MstarError) as e:
        ctx.integrate(m, x, v, 0.0, 1.0, M.params(k_fix=1))
    assert e.value.code == M.E_INVAL
    xg, vg, rc, st = ctx.integrate(m, x, v, 0.0, 10.0, M.params(max_steps=6), allow=(M.E_MAXSTEPS,))
    assert rc == M.E_MAXSTEPS and st["steps_accepted"] + st["steps_rejected"] == 6
    assert 0 <= st["t_reached"] < 10 and np.all(np.isfinite(xg))
    xg, vg, rc, st = ctx.integrate(m, x, v, 0.0, 1.0, M.params(eta=1e-30, max_halvings=2), allow=(M.E_NOCONV,))
    assert rc == M.E_NOCONV


def test_oversized_first_step_recovers(ctx, orc, M):
    """Sec. 2.3 failure handling forced from the host: a first step spanning
    the whole interval (q_first = 1e6, clipped to t_end) fails the error test
    and is halved until it converges; the run then ends at t_end with the
    energy kept at the tolerance level."""
    m, x, v = ics.plummer(16, 7)
    say("oversized first step")
    xg, vg, rc, st = ctx.integrate(m, x, v, 0.0, 2.0, M.params(eta=1e-12, q_first=1e6))
    assert rc == 0 and st["steps_rejected"] >= 5
    assert abs(st["t_reached"] - 2.0) <= 1e-14 * 2.0
    d0, d1 = orc.diagnostics(m, x, v), orc.diagnostics(m, xg, vg)
    assert abs((d1["E"] - d0["E"]) / d0["E"]) <= 1e-13


def test_workspace_reuse_across_sizes(ctx, orc, M):
    """Calls on one context with shrinking and growing N give the same result
    as on a fresh context (regression: stale start-slot increments)."""
    m, x, v = ics.plummer(48, 11)
    say("workspace reuse")
    fresh = M.Context(0)
    want = fresh.integrate(m, x, v, 0.0, 0.05)
    fresh.close()
    big = ics.plummer(700, 12)
    ctx.integrate(*big, 0.0, 1e-3)
    got = ctx.integrate(m, x, v, 0.0, 0.05)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_device_pointers(ctx, orc, M):
    import torch
    m, x, v = ics.plummer(64, 5)
    say("device pointers")
    mt = torch.tensor(m, device="cuda")
    xt = torch.tensor(x, device="cuda")
    vt = torch.tensor(v, device="cuda")
    xg, vg, rc, st = ctx.integrate(mt, xt, vt, 0.0, 0.05, M.params(eta=1e-12))
    xh, vh, rch, sth = ctx.integrate(m, x, v, 0.0, 0.05, M.params(eta=1e-12))
    assert np.array_equal(xg.cpu().numpy(), xh) and np.array_equal(vg.cpu().numpy(), vh)
