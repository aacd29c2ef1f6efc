"""GPU replay, force Hessian-vector product and adjoint vs the oracle, through the C ABI.

* force_hvp: dot-product test against the oracle's force tangent,
  <J u, w> = <u, J^T w>, and symmetry of the potential's Hessian
  diag(m) J (to 1e-12 relative).
* replay: the GPU's Cartesian replay and the oracle's MST replay evaluate the
  same map; end states agree to 1e-10 over short records.
* adjoint: dot-product test against the oracle TLM on random directions,
  <lambda, J delta> = <J^T lambda, delta> (1e-9 relative), central
  differences of the GPU replay (1e-6), and bitwise independence of the
  checkpoint interval and of the store limit (the recomputation is
  deterministic).  The GPU and the
  oracle linearise around their own trajectories, which differ by rounding
  that the dynamics stretches by the same factor G as the tangents; the
  mismatch of the dot products stays ~1e-12 while G <= 1e3 and grows to
  ~1e-8 at G ~ 1e4-1e5 (measured).  The comparisons therefore run on records
  whose stretch factor is at most ~1e3; longer records are checked for
  determinism and cost, and their mismatch is reported.
* autograd: torch gradients through paper_2001_03180_amd.autograd.integrate
  equal the direct adjoint call, and the gradient of the relative energy
  error matches central differences.
"""
import sys
import time

import numpy as np
import pytest

import ics

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-adj] {msg}", flush=True)
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


def record(orc, m, x, v, t_end, k, eta=1e-12):
    p = orc.params(eta=eta)
    xs, vs, rc, st, H, par = orc.integrate_rec(m, x, v, 0.0, t_end, k, p)
    assert rc == 0
    return H, par


@pytest.mark.parametrize("n", [257, 1000])
def test_force_hvp_dot_product_and_symmetry(ctx, orc, M, n):
    m, x, v = ics.plummer_with_central_mass(n - 1, 501)
    rng = np.random.default_rng(n)
    u, w = rng.standard_normal((2, n, 3))
    say(f"force_hvp n={n}")
    Jtw = ctx.force_hvp(m, x, w)
    _, _, Ju, _ = orc.force_tlm(m, x, u[None])
    lhs, rhs = np.sum(Ju[0] * w), np.sum(u * Jtw)
    scale = np.linalg.norm(Ju[0]) * np.linalg.norm(w)
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)
    Hw = ctx.force_hvp(m, x, m[:, None] * w)
    Hu = ctx.force_hvp(m, x, m[:, None] * u)
    s1, s2 = np.sum(u * Hw), np.sum(w * Hu)
    assert abs(s1 - s2) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(Hw)


@pytest.mark.parametrize("case", ["plummer32", "plummer256_bh"])
def test_replay_matches_oracle_replay(ctx, orc, M, case):
    if case == "plummer32":
        m, x, v = ics.plummer(32, 101)
        H, par = record(orc, m, x, v, 0.1, 1000)
    else:
        m, x, v, _ = ics.workload("plummer256_bh")
        H, par = record(orc, m, x, v, 10.0, 40)
    say(f"replay {case}: {len(H)} steps")
    xo, vo, to = orc.replay(m, x, v, 0.0, H, par, orc.params(eta=1e-12))
    xg, vg, tg = ctx.replay(m, x, v, 0.0, H)
    xg2, vg2, tg2 = ctx.replay(m, x, v, 0.0, H)
    assert np.array_equal(xg, xg2) and np.array_equal(vg, vg2) and tg == tg2
    R = np.abs(xo - (m[:, None] * xo).sum(0) / m.sum()).max()
    Vs = np.abs(vo - (m[:, None] * vo).sum(0) / m.sum()).max()
    assert np.abs(xg - xo).max() <= 1e-10 * R and np.abs(vg - vo).max() <= 1e-10 * Vs
    # t sums the extrapolated time increments; the extrapolation weights add
    # up to |c| ~ 1.2e2 in magnitude, so each step's rounding (~1e-16 of dt)
    # reaches ~1e-14 of it: 1e-12 of t over these records
    assert abs(tg - to) <= 1e-12 * abs(to)


def _adjoint_vs_tlm(ctx, orc, m, x, v, H, nd, seed, ce=50):
    n = len(m)
    rng = np.random.default_rng(seed)
    gx, gv = rng.standard_normal((2, n, 3))
    gt = float(rng.standard_normal())
    t0 = time.perf_counter()
    ax, av = ctx.replay_adjoint(m, x, v, 0.0, H, gx, gv, gt, ce)
    t_adj = time.perf_counter() - t0
    dx, dv = rng.standard_normal((2, nd, n, 3))
    t0 = time.perf_counter()
    _, _, _, Dx, Dv, Dt = orc.replay_tlm(m, x, v, 0.0, H, dx, dv, orc.params(eta=1e-12))
    t_tlm = time.perf_counter() - t0
    worst = 0.0
    for q in range(nd):
        lhs = np.sum(gx * Dx[q]) + np.sum(gv * Dv[q]) + gt * Dt[q]
        rhs = np.sum(ax * dx[q]) + np.sum(av * dv[q])
        scale = (np.linalg.norm(gx) * np.linalg.norm(Dx[q]) + np.linalg.norm(gv) * np.linalg.norm(Dv[q]) +
                 abs(gt * Dt[q]))
        worst = max(worst, abs(lhs - rhs) / scale)
    return worst, t_adj, t_tlm, (gx, gv, gt, ax, av)


def test_adjoint_dot_product_vs_oracle_tlm(ctx, orc, M):
    m, x, v = ics.plummer_with_central_mass(63, 7)
    H, par = record(orc, m, x, v, 10.0, 80)
    say(f"adjoint vs TLM: N={len(m)}, {len(H)} steps, 8 directions")
    worst, t_adj, t_tlm, _ = _adjoint_vs_tlm(ctx, orc, m, x, v, H, 8, 3, ce=16)
    say(f"worst relative dot-product mismatch {worst:.2e} (adjoint {t_adj:.2f} s, TLM {t_tlm:.2f} s)")
    assert worst <= 1e-9


def test_adjoint_checkpoint_interval_is_bitwise_irrelevant(ctx, orc, M):
    m, x, v = ics.plummer(40, 21)
    H, par = record(orc, m, x, v, 10.0, 37)
    rng = np.random.default_rng(2)
    gx, gv = rng.standard_normal((2, 40, 3))
    ref = ctx.replay_adjoint(m, x, v, 0.0, H, gx, gv, 0.3, 1)
    for ce in (2, 7, 36, 37, 100):
        say(f"checkpoint every {ce}")
        out = ctx.replay_adjoint(m, x, v, 0.0, H, gx, gv, 0.3, ce)
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])


def test_adjoint_store_limit_is_bitwise_irrelevant(ctx, orc, M):
    """Store limits below two segments' substep states split each segment into
    blocks recomputed from its step states (one step per block at the
    smallest limit, ragged blocks of two or three steps in between); the
    gradient stays the same to the bit, masses included."""
    m, x, v = ics.plummer(40, 21)
    H, par = record(orc, m, x, v, 10.0, 37)
    rng = np.random.default_rng(3)
    gx, gv = rng.standard_normal((2, 40, 3))
    ref = ctx.replay_adjoint(m, x, v, 0.0, H, gx, gv, 0.3, 1, with_mass=True)
    step_bytes = 32 * (2 * 8 * 8 + 3 * 8) * 40
    try:
        for limit, ce in ((1, 7), (6 * step_bytes, 7), (6 * step_bytes, 37), (1, 100)):
            say(f"store limit {limit} B, checkpoint every {ce}")
            ctx.adjoint_store_limit(limit)
            out = ctx.replay_adjoint(m, x, v, 0.0, H, gx, gv, 0.3, ce, with_mass=True)
            for a, b in zip(out, ref):
                assert np.array_equal(a, b)
    finally:
        ctx.adjoint_store_limit(0)
    with pytest.raises(M.MstarError):
        ctx.adjoint_store_limit(-1)


def test_adjoint_vs_finite_differences_of_replay(ctx, orc, M):
    m, x, v = ics.plummer(32, 101)
    H, par = record(orc, m, x, v, 10.0, 60)
    rng = np.random.default_rng(5)
    gx, gv = rng.standard_normal((2, 32, 3))
    ax, av = ctx.replay_adjoint(m, x, v, 0.0, H, gx, gv, 0.0, 20)
    say("finite differences of the GPU replay")

    def f(dx, dv, s):
        xe, ve, _ = ctx.replay(m, x + s * dx, v + s * dv, 0.0, H)
        return np.sum(gx * xe) + np.sum(gv * ve)

    # The map stretches perturbations by ~1e3-1e4 over this record, so its
    # higher derivatives are large: central differences at h and h/2 are
    # combined (Richardson) to cancel the h^2 term, with h small enough that
    # the h^4 term is negligible and large enough that rounding (~1e-12 of
    # the objective) stays below 1e-6 of the derivative.
    h = 1e-7
    for q in range(4):
        dx, dv = rng.standard_normal((2, 32, 3))
        d1 = (f(dx, dv, h) - f(dx, dv, -h)) / (2 * h)
        d2 = (f(dx, dv, h / 2) - f(dx, dv, -h / 2)) / h
        fd = (4 * d2 - d1) / 3
        ad = np.sum(ax * dx) + np.sum(av * dv)
        assert abs(fd - ad) <= 1e-6 * (abs(ad) + np.linalg.norm(ax) + np.linalg.norm(av)), (q, fd, ad)


def test_autograd_device_path_matches_host_path(ctx, M):
    """CUDA tensors go through the library's device-pointer path in both the
    forward and the backward pass; the results equal the host path's bit for
    bit and stay on the device."""
    import torch
    from paper_2001_03180_amd import autograd as AG
    m, x, v = ics.plummer_with_central_mass(31, 9)
    n = len(m)
    res = {}
    for dev in ("cpu", "cuda"):
        x0 = torch.tensor(x, device=dev, requires_grad=True)
        v0 = torch.tensor(v, device=dev, requires_grad=True)
        xs, vs, ts = AG.integrate(x0, v0, m, 0.0, 10.0, max_accepted=60, ctx=ctx, eta=1e-12, checkpoint_every=20)
        J = xs[n - 1].sum() + 0.5 * vs[0].sum() + ts
        gx, gv = torch.autograd.grad(J, (x0, v0))
        assert xs.device.type == dev and gx.device.type == dev
        res[dev] = [t.detach().cpu().numpy() for t in (xs, vs, ts, gx, gv)]
    for a, b in zip(res["cpu"], res["cuda"]):
        assert np.array_equal(a, b)


def test_autograd_function(ctx, orc, M):
    import torch
    from paper_2001_03180_amd import autograd as AG
    m, x, v = ics.plummer_with_central_mass(31, 9)
    n = len(m)
    x0 = torch.tensor(x, requires_grad=True)
    v0 = torch.tensor(v, requires_grad=True)
    say("autograd: central-mass position and energy error")
    xs, vs, ts = AG.integrate(x0, v0, m, 0.0, 10.0, max_accepted=80, ctx=ctx, eta=1e-12, checkpoint_every=25)
    J1 = xs[n - 1].sum()
    gx, gv = torch.autograd.grad(J1, (x0, v0))
    H = ctx.integrate_record(m, x, v, 0.0, 10.0, 80)[4]
    seed = np.zeros((n, 3))
    seed[n - 1] = 1.0
    ax, av = ctx.replay_adjoint(m, x, v, 0.0, H, seed, np.zeros((n, 3)), 0.0, 25)
    assert np.array_equal(gx.numpy(), ax) and np.array_equal(gv.numpy(), av)

    mt = torch.tensor(m)

    def energy(xx, vv):
        vc = vv - (mt[:, None] * vv).sum(0) / mt.sum()
        T = 0.5 * (mt * (vc * vc).sum(1)).sum()
        d = xx[:, None, :] - xx[None, :, :]
        r = torch.sqrt((d * d).sum(-1) + torch.eye(n, dtype=torch.float64))
        U = 0.5 * ((mt[:, None] * mt[None, :]) / r * (1 - torch.eye(n, dtype=torch.float64))).sum()
        return T - U

    x0.grad = None
    xs, vs, ts = AG.integrate(x0, v0, m, 0.0, 10.0, max_accepted=80, ctx=ctx, eta=1e-12)
    J2 = (energy(xs, vs) - energy(x0, v0)) / energy(x0, v0)
    g2x, g2v = torch.autograd.grad(J2, (x0, v0))
    rng = np.random.default_rng(8)
    h = 1e-6
    gE0 = torch.autograd.grad(energy(x0, v0), (x0, v0))
    scale = float(torch.cat([gE0[0].flatten(), gE0[1].flatten()]).norm()) / abs(float(energy(x0, v0).detach()))
    for q in range(3):
        dx, dv = rng.standard_normal((2, n, 3))

        def j2(s):
            xa, va = x + s * dx, v + s * dv
            xe, ve, _ = ctx.replay(m, xa, va, 0.0, H)
            Ea = float(energy(torch.tensor(xa), torch.tensor(va)))
            Eb = float(energy(torch.tensor(xe), torch.tensor(ve)))
            return (Eb - Ea) / Ea

        fd = (j2(h) - j2(-h)) / (2 * h)
        ad = float((g2x * torch.tensor(dx)).sum() + (g2v * torch.tensor(dv)).sum())
        # J2 is a difference of O(1) terms: compare in units of |grad E0| / |E0|
        assert abs(fd - ad) <= 1e-5 * scale * np.sqrt(np.sum(dx * dx) + np.sum(dv * dv)), (q, fd, ad)


def test_c5_workload_adjoint(ctx, orc, M):
    """N=256 Plummer + central mass 0.01, 1000 accepted GBS steps recorded by the
    GPU integrator, checkpoints every 50.  The gradient of the central mass's
    end position is compared with the oracle TLM over the first 200 steps
    (stretch factor ~7e2); over all 1000 steps (stretch ~1e12, past the
    predictability horizon) the adjoint is checked for determinism across
    checkpoint intervals and its cost and TLM mismatch are reported."""
    m, x, v, _ = ics.workload("plummer256_bh")
    n = len(m)
    t0 = time.perf_counter()
    xs, vs, rc, st, H = ctx.integrate_record(m, x, v, 0.0, 1e9, 1000, M.params(eta=1e-12))
    t_fwd = time.perf_counter() - t0
    assert len(H) == 1000
    say(f"C5 forward: 1000 accepted steps in {t_fwd:.2f} s (t = {st['t_reached']:.4f})")
    rng = np.random.default_rng(501)
    dx, dv = rng.standard_normal((2, 2, n, 3))
    _, _, _, Dx, Dv, Dt = orc.replay_tlm(m, x, v, 0.0, H[:200], dx, dv, orc.params(eta=1e-12))
    for c in range(3):
        seed = np.zeros((n, 3))
        seed[n - 1, c] = 1.0
        ax, av = ctx.replay_adjoint(m, x, v, 0.0, H[:200], seed, np.zeros((n, 3)), 0.0, 50)
        for q in range(2):
            lhs = Dx[q, n - 1, c]
            rhs = np.sum(ax * dx[q]) + np.sum(av * dv[q])
            scale = np.linalg.norm(ax) * np.linalg.norm(dx[q]) + np.linalg.norm(av) * np.linalg.norm(dv[q])
            assert abs(lhs - rhs) <= 1e-9 * scale, (c, q, lhs, rhs)
    seed = np.zeros((n, 3))
    seed[n - 1, 0] = 1.0
    t0 = time.perf_counter()
    ax, av = ctx.replay_adjoint(m, x, v, 0.0, H, seed, np.zeros((n, 3)), 0.0, 50)
    t_adj = time.perf_counter() - t0
    bx, bv = ctx.replay_adjoint(m, x, v, 0.0, H, seed, np.zeros((n, 3)), 0.0, 1000)
    assert np.array_equal(ax, bx) and np.array_equal(av, bv)
    say(f"C5 adjoint over 1000 steps: {t_adj:.2f} s = {t_adj / t_fwd:.2f} x the forward integration")
    _, _, _, Ex, Ev, _ = orc.replay_tlm(m, x, v, 0.0, H, dx[:1], dv[:1], orc.params(eta=1e-12))
    lhs, rhs = Ex[0, n - 1, 0], np.sum(ax * dx[0]) + np.sum(av * dv[0])
    growth = np.sqrt(np.sum(Ex[0] ** 2) + np.sum(Ev[0] ** 2)) / np.sqrt(np.sum(dx[0] ** 2) + np.sum(dv[0] ** 2))
    say(f"C5 1000 steps: stretch factor {growth:.1e}, adjoint vs TLM relative mismatch "
        f"{abs(lhs - rhs) / max(abs(lhs), 1e-300):.1e} (reported only)")
