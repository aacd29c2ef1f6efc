"""Batched small systems (one persistent launch) vs the CPU oracle, through the C ABI.

Each system of a batch is integrated exactly as the single-system driver
does; the oracle integrates the same systems one by one.  Tolerances: end
positions 1e-10 of the system's extent, velocities 1e-10 of the velocity
spread or, where a step decision flipped, the oracle's own accuracy
(check_vs_oracle); t_reached to 2e-14 t_end; step counts within the drift
that follows a flipped decision (check_counts).  Launch shapes (tile width,
the N cut between whole-workgroup and single-wave systems, workgroups per
CU, graph or plain launch) do not change a single bit of the result:
zero-padded lanes add exact zeros to every butterfly sum, and every per-body
quantity is computed by the same instruction sequence.
"""
import math
import sys

import numpy as np
import pytest

import ics

pytestmark = pytest.mark.gpu

T_SHORT = 1e-3      # horizon of the small parity batches
T_FULL = 1e-2       # horizon of the full 4096-system workload


def say(msg):
    print(f"[gpu-batch] {msg}", flush=True)
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


def sub_batch(off, m, x, v, idx):
    """Systems idx of a packed batch, repacked."""
    sizes = np.diff(off)[idx]
    o2 = np.zeros(len(idx) + 1, dtype=np.int64)
    o2[1:] = np.cumsum(sizes)
    rows = np.concatenate([np.arange(off[s], off[s + 1]) for s in idx])
    return o2, m[rows].copy(), x[rows].copy(), v[rows].copy()


@pytest.fixture(scope="module")
def small():
    """40 systems of the 4096-system workload (mixed N, triples included)."""
    off, m, x, v = ics.batch_subsystems()
    idx = list(range(40))
    return sub_batch(off, m, x, v, idx)


def rel_err(xg, vg, xo, vo, m):
    rc = (m[:, None] * xo).sum(0) / m.sum()
    vc = (m[:, None] * vo).sum(0) / m.sum()
    return np.abs(xg - xo).max() / np.abs(xo - rc).max(), np.abs(vg - vo).max() / np.abs(vo - vc).max()


def check_vs_oracle(orc, off, m, x, v, xg, vg, st, t_end, systems, eta=1e-12):
    """End states of `systems` against the oracle.

    Positions agree to 1e-10 of the system's extent.  Velocities agree to
    1e-10 of the velocity spread, or, where a flipped step decision
    (check_counts) has put a phase error of the innermost orbit between the
    two runs, to within the oracle's own integration error: the GPU error
    against a reference run of the oracle at eta = 1e-14 may not exceed four
    times the oracle's error against it (plus 1e-12).  Returns
    (worst error vs the oracle, systems that needed the reference)."""
    worst, via_ref = 0.0, []
    for s in systems:
        o, e = int(off[s]), int(off[s + 1])
        ms, xs, vs = m[o:e], x[o:e], v[o:e]
        xo, vo, rco, sto = orc.integrate(ms, xs, vs, 0.0, t_end, orc.params(eta=eta))
        assert st["status"][s] == rco == 0, (s, st["status"][s], rco)
        check_counts(st, s, sto)
        assert abs(st["t_reached"][s] - sto["t_reached"]) <= 2e-14 * abs(t_end), s
        ex, ev = rel_err(xg[o:e], vg[o:e], xo, vo, ms)
        worst = max(worst, ex, ev)
        assert ex <= 1e-10, (s, e - o, ex)
        if ev > 1e-10:
            xr, vr, rcr, _ = orc.integrate(ms, xs, vs, 0.0, t_end, orc.params(eta=1e-14))
            assert rcr == 0
            gx, gv = rel_err(xg[o:e], vg[o:e], xr, vr, ms)
            ox, ov = rel_err(xo, vo, xr, vr, ms)
            say(f"system {s} N={e - o}: gpu vs oracle {ev:.1e}; vs reference gpu {gv:.1e}, oracle {ov:.1e}")
            assert gx <= 4 * ox + 1e-12 and gv <= 4 * ov + 1e-12, (s, gx, ox, gv, ov)
            via_ref.append(s)
    return worst, via_ref


def check_counts(st, s, sto):
    """Step counts agree up to the drift that follows a flipped decision.

    The error measure of a step is |T_kk - T_k-1,k-1| / |S|, a difference
    of two extrapolated values whose rounding noise (~1e-14 of |S|) is a few
    per cent of eta = 1e-12; a step whose measure lies that close to eta can
    be accepted by one correct implementation and rejected by another, and
    the step sequences differ from there on."""
    for k in ("steps_accepted", "steps_rejected"):
        a, b = int(st[k][s]), int(sto[k])
        assert abs(a - b) <= max(5, 0.1 * b), (s, k, a, b)


def test_batch_parity_small(ctx, orc, M, small):
    off, m, x, v = small
    say(f"batch of {len(off) - 1} systems, t_end={T_SHORT}")
    xg, vg, st = ctx.integrate_batch(off, m, x, v, T_SHORT, p=M.params(eta=1e-12))
    worst, via_ref = check_vs_oracle(orc, off, m, x, v, xg, vg, st, T_SHORT, range(len(off) - 1))
    say(f"worst relative state error vs oracle {worst:.2e}; checked against the reference: {via_ref}")
    assert len(via_ref) <= 8


def test_batch_matches_single_system_path(ctx, M, small):
    """The batch kernel and the multi-launch single-system path agree."""
    off, m, x, v = small
    xg, vg, st = ctx.integrate_batch(off, m, x, v, T_SHORT, p=M.params(eta=1e-12))
    for s in (0, 3, 7, 11):
        o, e = int(off[s]), int(off[s + 1])
        say(f"single-system path, system {s} (N={e - o})")
        xs, vs, rc, sts = ctx.integrate(m[o:e], x[o:e], v[o:e], 0.0, T_SHORT, M.params(eta=1e-12))
        assert rc == 0
        check_counts(st, s, sts)
        ex, ev = rel_err(xg[o:e], vg[o:e], xs, vs, m[o:e])
        assert ex <= 1e-10 and ev <= 1e-10, (s, ex, ev)


def test_launch_shapes_bitwise_identical(ctx, M, small):
    off, m, x, v = small
    ref = None
    shapes = [(0, 0, 0, 0), (16, 16, 0, 1), (32, 32, 1, 1), (32, 16, 2, 0), (64, 64, 0, 1), (64, 32, 1, 0)]
    try:
        for wl, wmax, per, graph in shapes:
            ctx.set_batch_config(8, wave_lanes=wl, wave_max_n=wmax, wgs_per_cu=per, use_graph=graph)
            say(f"shape wave_lanes={wl} wave_max_n={wmax} wgs_per_cu={per} graph={graph}")
            out = ctx.integrate_batch(off, m, x, v, T_SHORT, p=M.params(eta=1e-12))
            if ref is None:
                ref = out
                continue
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])
            assert np.array_equal(out[2], ref[2])
    finally:
        ctx.set_batch_config(8, wave_lanes=16, wave_max_n=16, wgs_per_cu=0, use_graph=1)


def test_graph_replays(ctx, M, small):
    """Replays of the captured graph, with other GPU work in between, match a plain launch."""
    import torch
    off, m, x, v = small
    ctx.set_batch_config(8, use_graph=0)
    ref = ctx.integrate_batch(off, m, x, v, T_SHORT, p=M.params(eta=1e-12))
    ctx.set_batch_config(8, use_graph=1)
    for r in range(3):
        say(f"graph replay {r}")
        out = ctx.integrate_batch(off, m, x, v, T_SHORT, p=M.params(eta=1e-12))
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()   # eager work between replays
        torch.cuda.synchronize()
        assert math.isfinite(float(junk))
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])
        assert np.array_equal(out[2], ref[2])


def test_device_pointers(ctx, M, small):
    import torch
    off, m, x, v = small
    ref = ctx.integrate_batch(off, m, x, v, T_SHORT, p=M.params(eta=1e-12))
    dm = torch.tensor(m, device="cuda")
    dx = torch.tensor(x, device="cuda")
    dv = torch.tensor(v, device="cuda")
    say("device pointers")
    xg, vg, st = ctx.integrate_batch(off, dm, dx, dv, T_SHORT, p=M.params(eta=1e-12))
    assert np.array_equal(xg.cpu().numpy(), ref[0]) and np.array_equal(vg.cpu().numpy(), ref[1])
    assert np.array_equal(st, ref[2])
    assert np.array_equal(dx.cpu().numpy(), x)   # the binding integrates a copy


def test_kepler_closed_form(ctx, M):
    from tests import kepler
    es = [0.0, 0.5, 0.9, 0.99]
    parts = [ics.kepler_two_body(0.5, 0.5, 1.0, e, seed=3 + k) for k, e in enumerate(es)]
    off = np.arange(0, 2 * len(es) + 1, 2, dtype=np.int64)
    m = np.concatenate([p[0] for p in parts])
    x = np.concatenate([p[1] for p in parts])
    v = np.concatenate([p[2] for p in parts])
    tend = 3.3 * 2 * math.pi
    say("kepler batch")
    xg, vg, st = ctx.integrate_batch(off, m, x, v, tend, p=M.params(eta=1e-12))
    for s in range(len(es)):
        o = 2 * s
        assert st["status"][s] == 0 and abs(st["t_reached"][s] - tend) <= 1e-14 * tend
        r, u = kepler.propagate(1.0, x[o + 1] - x[o], v[o + 1] - v[o], st["t_reached"][s])
        err = np.abs((xg[o + 1] - xg[o]) - r).max() / np.linalg.norm(r)
        assert err < 5e-12 * (10.0 if es[s] > 0.95 else 1.0), (es[s], err)


def test_per_system_errors(ctx, M, small):
    """Bad systems get their own status; the other systems are unaffected."""
    off, m, x, v = small
    idx = [0, 1, 2, 3, 4]
    o5, m5, x5, v5 = sub_batch(off, m, x, v, idx)
    ref = ctx.integrate_batch(o5, m5, x5, v5, T_SHORT, p=M.params(eta=1e-12))
    mb, xb, vb = m5.copy(), x5.copy(), v5.copy()
    xb[o5[1] + 1] = xb[o5[1] + 2]          # coincident bodies in system 1
    vb[o5[2] + 1, 2] = np.nan              # non-finite velocity in system 2
    mb[o5[3] + 1] = 0.0                    # zero mass in system 3
    say("per-system errors")
    xg, vg, st = ctx.integrate_batch(o5, mb, xb, vb, T_SHORT, p=M.params(eta=1e-12))
    assert list(st["status"]) == [M.OK, M.E_COINCIDENT, M.E_NONFINITE, M.E_INVAL, M.OK]
    for s in (0, 4):
        sl = slice(o5[s], o5[s + 1])
        assert np.array_equal(xg[sl], ref[0][sl]) and np.array_equal(vg[sl], ref[1][sl])
    for s in (1, 2, 3):   # untouched
        sl = slice(o5[s], o5[s + 1])
        assert np.array_equal(xg[sl], xb[sl], equal_nan=True)
    say("max_steps")
    xg, vg, st = ctx.integrate_batch(o5, m5, x5, v5, 1.0, p=M.params(eta=1e-12, max_steps=5))
    for s in range(5):
        if st["status"][s] == M.E_MAXSTEPS:
            assert st["steps_accepted"][s] + st["steps_rejected"][s] == 5
            assert 0.0 <= st["t_reached"][s] < 1.0
        else:
            assert st["status"][s] == M.OK
    assert (st["status"] == M.E_MAXSTEPS).sum() >= 3
    assert np.all(np.isfinite(xg))


def test_call_validation(ctx, M, small):
    off, m, x, v = small
    say("validation")
    cases = [
        (dict(p=M.params(k_fix=9)), M.E_UNSUPPORTED),
        (dict(p=M.params(beta=1.0)), M.E_UNSUPPORTED),
        (dict(p=M.params(n_d=3)), M.E_UNSUPPORTED),
        (dict(t_end=0.0), M.E_INVAL),
    ]
    for kw, code in cases:
        args = dict(t_end=T_SHORT, p=M.params())
        args.update(kw)
        with pytest.raises(M.MstarError) as e:
            ctx.integrate_batch(off, m, x, v, args["t_end"], p=args["p"])
        assert e.value.code == code, kw
    big_m, big_x, big_v = ics.plummer(65, 5)
    with pytest.raises(M.MstarError) as e:
        ctx.integrate_batch(np.array([0, 65]), big_m, big_x, big_v, T_SHORT)
    assert e.value.code == M.E_UNSUPPORTED
    with pytest.raises(M.MstarError) as e:
        ctx.integrate_batch(np.array([0, 1, 3]), m[:3], x[:3], v[:3], T_SHORT)
    assert e.value.code == M.E_INVAL
    with pytest.raises(M.MstarError) as e:
        ctx.set_batch_config(8, wave_lanes=24)
    assert e.value.code == M.E_INVAL


def test_autotune(ctx, M):
    off, m, x, v = ics.batch_subsystems()
    o2, m2, x2, v2 = sub_batch(off, m, x, v, list(range(256)))
    say("autotune on 256 systems")
    before = ctx.integrate_batch(o2, m2, x2, v2, T_SHORT, p=M.params(eta=1e-12))
    best = ctx.batch_autotune(o2, m2, x2, v2, 2e-4, p=M.params(eta=1e-12))
    say(f"autotune choice {best}")
    assert best["wave_lanes"] in (0, 16, 32, 64) and 0 <= best["wave_max_n"] <= best["wave_lanes"]
    assert best["wgs_per_cu"] >= 1 and best["kernel_ms"] > 0 and best["use_graph"] == 1
    assert ctx.batch_config(8) == best
    after = ctx.integrate_batch(o2, m2, x2, v2, T_SHORT, p=M.params(eta=1e-12))
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[2], after[2])
    ctx.set_batch_config(8, wave_lanes=16, wave_max_n=16, wgs_per_cu=0, use_graph=1)


def test_full_workload_sampled(ctx, orc, M):
    """The 4096-system workload at its full horizon (about 50 periods of the
    innermost orbits) in the launch the benchmark times; sampled systems
    (largest, median-size, smallest, a triple) against the oracle as in
    check_vs_oracle, and energy conservation of every system."""
    off, m, x, v = ics.batch_subsystems()
    sizes = np.diff(off)
    say(f"full workload: {len(sizes)} systems, {off[-1]} bodies, t_end={T_FULL}")
    xg, vg, st = ctx.integrate_batch(off, m, x, v, T_FULL, p=M.params(eta=1e-12))
    assert np.all(st["status"] == M.OK), np.unique(st["status"], return_counts=True)
    assert np.all(np.abs(st["t_reached"] - T_FULL) <= 1e-14 * T_FULL)
    order = np.argsort(sizes, kind="stable")
    triple = int(np.nonzero(sizes == 3)[0][0])
    sample = [int(order[-1]), int(order[len(order) // 2]), int(order[0]), triple]
    say(f"oracle on systems {sample} (N={[int(sizes[s]) for s in sample]})")
    worst, via_ref = check_vs_oracle(orc, off, m, x, v, xg, vg, st, T_FULL, sample)
    say(f"worst relative state error vs oracle {worst:.2e}; checked against the reference: {via_ref}")
    dE = np.empty(len(sizes))
    for s in range(len(sizes)):
        o, e = int(off[s]), int(off[s + 1])
        E0 = orc.diagnostics(m[o:e], x[o:e], v[o:e])["E"]
        E1 = orc.diagnostics(m[o:e], xg[o:e], vg[o:e])["E"]
        dE[s] = abs((E1 - E0) / E0)
    say(f"|dE/E|: median {np.median(dE):.2e}, 99% {np.quantile(dE, 0.99):.2e}, max {dE.max():.2e}")
    assert dE.max() <= 1e-11
