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
quantity is computed by the same instruction sequence.  Replay mode
(check_replay) removes the step decisions: the oracle repeats the GPU's
recorded step lengths, and the end states are compared against the oracle's
own sensitivity to ulp-sized changes of its inputs and step lengths.
"""
import math
import sys

import numpy as np
import pytest

import ics

pytestmark = pytest.mark.gpu

T_SHORT = 1e-3      # horizon of the small parity batches
T_FULL = 1e-2       # horizon of the full 4096-system workload


def _replay_time_rel(k_fix=8):
    """Bound on |t_gpu - t_replay| / t_end when the oracle replays recorded steps.

    A step's time increment is the Neville-Aitken extrapolation to h -> 0
    (Sec. 2.3) of the division sums over n_k = 2k substeps; each sum carries
    at most (n_k + 2) u of relative rounding, and the extrapolation weights
    L_k of the sequence x_k = 1/n_k^2 (sum |L_k| = 119 at k_fix = 8) amplify
    it to sum_k |L_k| (n_k + 2) u of the step.  Nothing clips the replayed
    time to t_end, so two correct runs can differ by twice that, summed over
    the steps: about 4.1e-13 of the interval."""
    n = [2.0 * k for k in range(1, k_fix + 1)]
    x = [1.0 / (v * v) for v in n]
    L = [math.prod(xj / (xj - xi) for j, xj in enumerate(x) if j != i) for i, xi in enumerate(x)]
    return 2.0 * sum(abs(l) * (v + 2.0) for l, v in zip(L, n)) * np.finfo(float).eps / 2


REPLAY_TIME_REL = _replay_time_rel()


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


def _ulp_sensitivity(orc, ms, xs, vs, H, xr, vr, ts, p):
    """How far the oracle's own replay moves under ulp-sized perturbations of
    two kinds: one input coordinate moved by one ulp (a position, then a
    velocity), and every step length moved by one ulp up or down at random
    (seeded; two draws).  The second kind stands for what two correct
    implementations do differently at every step: each step's extrapolated
    increments carry rounding amplified by the extrapolation weights, and in
    well-conditioned systems (a planet-like system of 38 steps) these
    per-step differences, not the start state's, dominate the end.  Returns
    the largest relative end-state change, the largest change of the end
    energy relative to the initial energy, and the largest change of the time
    after any step (ts: the unperturbed times).  Close eccentric pairs
    amplify the state change to ~1e-11 over 1e-3 time units, mostly as a
    phase shift along their orbits; since the time runs slower near each
    pericentre, a phase shift moves the time after a step back and forth by
    an amount that is largest somewhere inside the run, not necessarily at
    its end."""
    n = len(ms)
    E0 = orc.diagnostics(ms, xs, vs)["E"]
    Er = orc.diagnostics(ms, xr, vr)["E"]
    ws, we, wt = 0.0, 0.0, 0.0
    for j in range(4):
        x2, v2, H2 = xs.copy(), vs.copy(), H
        if j == 0:
            x2[0, 0] = np.nextafter(x2[0, 0], np.inf)
        elif j == 1:
            v2[n // 2, 1] = np.nextafter(v2[n // 2, 1], np.inf)
        else:
            up = np.random.default_rng(j).integers(0, 2, len(H)) == 1
            H2 = np.where(up, np.nextafter(H, np.inf), np.nextafter(H, -np.inf))
        xp, vp, _, tp = orc.replay(ms, x2, v2, 0.0, H2, None, p, times=True)
        ws = max(ws, *rel_err(xp, vp, xr, vr, ms))
        we = max(we, abs((orc.diagnostics(ms, xp, vp)["E"] - Er) / E0))
        wt = max(wt, float(np.abs(tp - ts).max(initial=0.0)))
    return ws, we, wt


def check_replay(orc, off, m, x, v, xg, vg, st, H, t_end, systems, eta=1e-12, threads=16):
    """Replay mode (no step decisions): the oracle integrates each system with
    the GPU's recorded accepted step lengths and its own MST builds and
    rebuilds.  The two runs round differently at every step, so their end
    states can differ by what the replay map makes of ulp-level changes.
    Each system's state error may not exceed ten times the oracle's own
    change under ulp-sized perturbations (_ulp_sensitivity), with a
    floor of 1e-12 of the system's extent and velocity spread; the end
    energies (relative to the initial one) agree to ten times the energy
    change under the same perturbations, with a floor of 1e-13; the end
    times agree to ten times the largest time change under them after any
    step, with a floor of REPLAY_TIME_REL of the interval.  Returns per-system (state error,
    |dE/E| GPU, |dE/E| replay, state, energy and time sensitivities)."""
    import concurrent.futures as cf

    def one(s):
        o, e = int(off[s]), int(off[s + 1])
        ms, xs, vs = m[o:e], x[o:e], v[o:e]
        k = int(st["steps_accepted"][s])
        assert st["status"][s] == 0 and k <= H.shape[1], (s, st["status"][s], k)
        p = orc.params(eta=eta, nthreads=1)
        xr, vr, tr, ts = orc.replay(ms, xs, vs, 0.0, H[s, :k], None, p, times=True)
        ex, ev = rel_err(xg[o:e], vg[o:e], xr, vr, ms)
        E0 = orc.diagnostics(ms, xs, vs)["E"]
        dg = (orc.diagnostics(ms, xg[o:e], vg[o:e])["E"] - E0) / E0
        dr = (orc.diagnostics(ms, xr, vr)["E"] - E0) / E0
        return (s, max(ex, ev), dg, dr, tr - st["t_reached"][s]) + \
            _ulp_sensitivity(orc, ms, xs, vs, H[s, :k], xr, vr, ts, p)

    with cf.ThreadPoolExecutor(max_workers=threads) as pool:
        out = list(pool.map(one, systems))
    for s, err, dg, dr, dt, sens, sens_e, sens_t in out:
        assert err <= max(1e-12, 10.0 * sens), (s, err, sens)
        assert abs(dg - dr) <= max(1e-13, 10.0 * sens_e), (s, dg, dr, sens_e)
        assert abs(dt) <= max(REPLAY_TIME_REL * abs(t_end), 10.0 * sens_t), (s, dt, sens_t)
    return [(s, err, dg, dr, sens) for s, err, dg, dr, dt, sens, sens_e, sens_t in out]


def test_batch_parity_small(ctx, orc, M, small):
    """All 40 systems: replay mode (the batch kernel's arithmetic, free of
    step decisions, against the oracle's own rounding sensitivity), then
    free mode against the oracle's own integration: 1e-10 for every system whose accepted and rejected step
    counts equal the oracle's; where a decision differed, the difference
    is reported together with the size of the integration error itself."""
    off, m, x, v = small
    n_sys = len(off) - 1
    say(f"batch of {n_sys} systems, t_end={T_SHORT}, recording the accepted steps")
    xg, vg, st, H = ctx.integrate_batch_record(off, m, x, v, T_SHORT, 4096, p=M.params(eta=1e-12))
    xb, vb, stb = ctx.integrate_batch(off, m, x, v, T_SHORT, p=M.params(eta=1e-12))
    assert np.array_equal(xg, xb) and np.array_equal(vg, vb) and np.array_equal(st, stb)   # recording is passive
    rep = check_replay(orc, off, m, x, v, xg, vg, st, H, T_SHORT, range(n_sys))
    say(f"replay mode: worst state error {max(r[1] for r in rep):.2e} (worst error / ulp sensitivity "
        f"{max(r[1] / max(r[4], 1e-300) for r in rep):.2f}), worst |dE/E gpu - replay| "
        f"{max(abs(r[2] - r[3]) for r in rep):.2e}")
    flips = []
    for s in range(n_sys):
        o, e = int(off[s]), int(off[s + 1])
        xo, vo, rco, sto = orc.integrate(m[o:e], x[o:e], v[o:e], 0.0, T_SHORT, orc.params(eta=1e-12))
        assert rco == 0 and abs(st["t_reached"][s] - sto["t_reached"]) <= 2e-14 * T_SHORT
        ex, ev = rel_err(xg[o:e], vg[o:e], xo, vo, m[o:e])
        same = (st["steps_accepted"][s], st["steps_rejected"][s]) == (sto["steps_accepted"], sto["steps_rejected"])
        if same:
            assert ex <= 1e-10 and ev <= 1e-10, (s, ex, ev)
        else:
            flips.append(s)
            say(f"system {s} N={e - o}: steps gpu {st['steps_accepted'][s]}+{st['steps_rejected'][s]} oracle "
                f"{sto['steps_accepted']}+{sto['steps_rejected']}: free-mode difference {max(ex, ev):.1e}")
            assert ex <= 1e-10, (s, ex)
    say(f"free mode: {n_sys - len(flips)} of {n_sys} systems took the oracle's step sequence; flips {flips}")


def test_record_buffer_survives_growth(ctx, M, small):
    """A recording call, then calls on larger batches (the context grows its
    batch buffers), then a recording call again: the record buffer belongs to
    the recording calls alone and the repeated record is identical."""
    off, m, x, v = small
    o8, m8, x8, v8 = sub_batch(off, m, x, v, list(range(8)))
    p = M.params(eta=1e-12)
    first = ctx.integrate_batch_record(o8, m8, x8, v8, T_SHORT, 512, p=p)
    full = ics.batch_subsystems()
    for k in (300, 600):
        o2, m2, x2, v2 = sub_batch(*full, list(range(k)))
        ctx.integrate_batch(o2, m2, x2, v2, 2e-4, p=p)
    again = ctx.integrate_batch_record(o8, m8, x8, v8, T_SHORT, 512, p=p)
    for a, b in zip(first[:3], again[:3]):
        assert np.array_equal(a, b)
    H1, H2, acc = first[3], again[3], first[2]["steps_accepted"]
    assert np.array_equal(H1, H2, equal_nan=True)
    for s in range(len(acc)):   # recorded steps finite, the rest of each row NaN
        assert np.all(np.isfinite(H1[s, :acc[s]])) and np.all(np.isnan(H1[s, acc[s]:]))


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
        (dict(p=M.params(n_d=5)), M.E_UNSUPPORTED),
        (dict(p=M.params(k_fix=17)), M.E_INVAL),
        (dict(t_end=0.0), M.E_INVAL),
    ]
    for kw, code in cases:
        args = dict(t_end=T_SHORT, p=M.params())
        args.update(kw)
        with pytest.raises(M.MstarError) as e:
            ctx.integrate_batch(off, m, x, v, args["t_end"], p=args["p"])
        assert e.value.code == code, kw
    with pytest.raises(M.MstarError) as e:
        ctx.integrate_batch(np.array([0, 1, 3]), m[:3], x[:3], v[:3], T_SHORT)
    assert e.value.code == M.E_INVAL
    with pytest.raises(M.MstarError) as e:
        ctx.set_batch_config(8, wave_lanes=24)
    assert e.value.code == M.E_INVAL


def test_systems_beyond_the_kernel_use_the_single_system_driver(ctx, M):
    """Systems of more than 64 bodies in a batch are integrated by
    mstar_integrate's driver after the persistent launch: the same end state,
    statistics and recorded steps as separate mstar_integrate_record calls,
    bit for bit, next to the small systems of the same call (unchanged by the
    larger ones' presence), on host and device arrays; a bad large system gets
    its own status."""
    import torch
    sizes = [(5, 1), (100, 2), (12, 3), (257, 4)]
    parts = [ics.plummer_with_central_mass(n - 1, seed) for n, seed in sizes]
    off = np.concatenate([[0], np.cumsum([n for n, _ in sizes])]).astype(np.int64)
    m = np.concatenate([q[0] for q in parts])
    x = np.concatenate([q[1] for q in parts])
    v = np.concatenate([q[2] for q in parts])
    p = M.params(eta=1e-12)
    t_end = 0.01
    say("mixed batch: N = 5, 100, 12, 257")
    xb, vb, st, H = ctx.integrate_batch_record(off, m, x, v, t_end, 64, p=p)
    small_only = ctx.integrate_batch(np.array([0, 5]), m[:5], x[:5], v[:5], t_end, p=p)
    assert np.array_equal(xb[:5], small_only[0]) and np.array_equal(vb[:5], small_only[1])
    for s, (n, _) in enumerate(sizes):
        o, e = int(off[s]), int(off[s + 1])
        assert st["status"][s] == M.OK
        if n <= 64:
            continue
        xs, vs, rc, ss, Hs = ctx.integrate_record(m[o:e], x[o:e], v[o:e], 0.0, t_end, 10 ** 6, p)
        assert np.array_equal(xb[o:e], xs) and np.array_equal(vb[o:e], vs)
        assert st["steps_accepted"][s] == ss["steps_accepted"] and st["force_evals"][s] == ss["force_evals"]
        assert st["t_reached"][s] == ss["t_reached"]
        k = min(len(Hs), 64)
        assert np.array_equal(H[s, :k], Hs[:k]) and np.all(np.isnan(H[s, k:]))
    # device arrays
    T = lambda a: torch.tensor(a, device="cuda")
    xd, vd, std = ctx.integrate_batch(off, T(m), T(x), T(v), t_end, p=p)
    assert np.array_equal(xd.cpu().numpy(), xb) and np.array_equal(vd.cpu().numpy(), vb)
    # a large system with a zero mass: its own error, the others unaffected
    m2 = m.copy()
    m2[int(off[3]) + 7] = 0.0
    x2, v2, st2 = ctx.integrate_batch(off, m2, x, v, t_end, p=p)
    assert st2["status"][3] == M.E_INVAL and all(st2["status"][s] == M.OK for s in range(3))
    assert np.array_equal(x2[:int(off[3])], xb[:int(off[3])])
    # only large systems: nothing for the persistent kernel
    say("batch of large systems only: N = 100, 257")
    o3 = np.array([0, 100, 357], dtype=np.int64)
    sl = np.r_[int(off[1]):int(off[2]), int(off[3]):int(off[4])]
    x3, v3, st3, H3 = ctx.integrate_batch_record(o3, m[sl], x[sl], v[sl], t_end, 64, p=p)
    assert np.array_equal(x3[:100], xb[int(off[1]):int(off[2])]) and np.array_equal(x3[100:], xb[int(off[3]):])
    assert np.array_equal(v3[:100], vb[int(off[1]):int(off[2])]) and np.array_equal(v3[100:], vb[int(off[3]):])
    assert np.array_equal(st3, st[[1, 3]])
    assert np.array_equal(H3, H[[1, 3]], equal_nan=True)
    before = ctx.batch_config(8)
    with pytest.raises(M.MstarError) as e:   # nothing for the autotuner to time
        ctx.batch_autotune(o3, m[sl], x[sl], v[sl], t_end, p=p)
    assert e.value.code == M.E_INVAL and ctx.batch_config(8) == before


@pytest.mark.parametrize("kw", [dict(k_fix=9), dict(beta=1.0), dict(n_d=3), dict(accept_rule=1)],
                         ids=["k_fix9", "ttl", "n_d3", "accept_rule1"])
def test_parameters_beyond_the_kernel_use_the_single_system_driver(ctx, M, small, kw):
    """Parameter sets the persistent kernel does not implement send every
    system of the call through mstar_integrate's driver: end states,
    statistics and recorded steps equal separate mstar_integrate_record calls
    bit for bit, on host and device arrays.  The autotuner, which times the
    kernel, refuses them."""
    import torch
    off, m, x, v = small
    o2, m2, x2, v2 = sub_batch(off, m, x, v, list(range(6)))
    p = M.params(eta=1e-12, **kw)
    say(f"batch with {kw}: {len(o2) - 1} systems")
    xb, vb, st, H = ctx.integrate_batch_record(o2, m2, x2, v2, T_SHORT, 32, p=p)
    for s in range(len(o2) - 1):
        o, e = int(o2[s]), int(o2[s + 1])
        xs, vs, rc, ss, Hs = ctx.integrate_record(m2[o:e], x2[o:e], v2[o:e], 0.0, T_SHORT, 10 ** 6, p)
        assert st["status"][s] == M.OK and rc == M.OK
        assert np.array_equal(xb[o:e], xs) and np.array_equal(vb[o:e], vs)
        for f in ("steps_accepted", "steps_rejected", "force_evals", "t_reached", "h_next"):
            assert st[f][s] == ss[f], f
        k = min(len(Hs), 32)
        assert np.array_equal(H[s, :k], Hs[:k]) and np.all(np.isnan(H[s, k:]))
    T = lambda a: torch.tensor(a, device="cuda")
    xd, vd, _ = ctx.integrate_batch(o2, T(m2), T(x2), T(v2), T_SHORT, p=p)
    assert np.array_equal(xd.cpu().numpy(), xb) and np.array_equal(vd.cpu().numpy(), vb)
    with pytest.raises(M.MstarError) as e:
        ctx.batch_autotune(o2, m2, x2, v2, T_SHORT, p=p)
    assert e.value.code == M.E_UNSUPPORTED


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
    # 64 systems spread over N (every 64th by size) and 8 hierarchical triples,
    # replayed by the oracle with the recorded step lengths
    xr, vr, str_, H = ctx.integrate_batch_record(off, m, x, v, T_FULL, 8192, p=M.params(eta=1e-12))
    assert np.array_equal(xr, xg) and np.array_equal(vr, vg)
    order = np.argsort(sizes, kind="stable")
    triples = [int(s) for s in np.nonzero(sizes == 3)[0][:8]]
    sample = sorted(set(int(order[k]) for k in range(0, len(order), 64)) | set(triples))
    say(f"oracle replay of {len(sample)} systems (N {int(sizes[sample].min())}..{int(sizes[sample].max())}, "
        f"{len(triples)} triples)")
    rep = check_replay(orc, off, m, x, v, xg, vg, st, H, T_FULL, sample)
    say(f"replay mode: worst state error {max(r[1] for r in rep):.2e} (worst error / ulp sensitivity "
        f"{max(r[1] / max(r[4], 1e-300) for r in rep):.2f}), worst |dE/E gpu - replay| "
        f"{max(abs(r[2] - r[3]) for r in rep):.2e}")
    dE = np.empty(len(sizes))
    for s in range(len(sizes)):
        o, e = int(off[s]), int(off[s + 1])
        E0 = orc.diagnostics(m[o:e], x[o:e], v[o:e])["E"]
        E1 = orc.diagnostics(m[o:e], xg[o:e], vg[o:e])["E"]
        dE[s] = abs((E1 - E0) / E0)
    say(f"|dE/E|: median {np.median(dE):.2e}, 99% {np.quantile(dE, 0.99):.2e}, max {dE.max():.2e}")
    assert dE.max() <= 1e-11
