"""Benchmark: FP64 pair interactions per second of the full MSTAR step at N=5000.

Workload (seeded, synthetic): Plummer sphere of 5000 equal-mass stars (total
mass 1, Henon units) with an embedded point-mass binary (2 x 0.005, a = 1e-3,
e = 0.9, random orientation) at its centre -> N_p = 5002 bodies; eta = 1e-13,
k_fix = 8, N_d = 2, LogH.  One "step" is one GBS step attempt of the
integrator: MST rebuild (after an accepted step), tree transforms, the start
force evaluation, all 8 substep divisions (72 force evaluations), Neville
extrapolation, error test and step control -- every row of the hot path.

The second half of the metric, batched small systems: 4096 independent
systems (N_p uniform in 3..64, central mass 1 + stars of 1e-5, 10% triples;
seed 401) integrated to t_end = 1e-2 at eta = 1e-12 in one persistent launch
(captured HIP graph) with the autotuned launch shape.  Reported as systems/s
with inputs resident in HBM (and with host copies), next to the per-system
loop of the same library (mstar_integrate, one system per call, a seeded
random sample of systems timed and scaled to the whole set) and to the CPU
oracle (one system per host thread, a seeded random sample).

The `adjoint` object: N=256 Plummer + central mass 0.01 (seed 501), 1000
accepted GBS steps at eta = 1e-12 recorded by the integrator; the gradient
of the central mass's end position (one component) with respect to all 6N
initial coordinates by the checkpointed adjoint (every 50 steps), timed
against the forward integration.

value = (force evaluations x N_p (N_p - 1)) / wall time of the timed steps,
inputs resident in HBM.  The roofline entry is the force kernel's algorithmic
FLOP rate (20 FP64 flops per directed pair) from HIP events around every
force launch during a repeat of the timed steps.  cpu_baseline times the CPU oracle (plain C,
OpenMP over i) on a bounded sample: one GBS step of the same state.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 pair-interactions/s at N=5000; batched subsystems/s vs per-system"
PEAK_FP64_TFLOPS = 78.6          # MI355X FP64 vector: 256 CU x 128 FLOP/clk x 2.4 GHz
FLOPS_PER_PAIR = 20
# VALU instructions per pair besides the hardware 1/sqrt, counted in the gfx950
# code of the two force kernels:
#  pairwise k_force, per directed pair: 3 differences, 3 for r^2, 5 for the
#  1/sqrt refinement, 3 for m/r and m/r^3, 4 accumulations = 18, one 1/sqrt;
#  mutual k_force_mut, per unordered pair: 3 + 3 + 5, 2 for r^-3, 2 for the two
#  masses' factors, 1 for phi, 3 + 3 accumulations into both bodies = 22 FP64,
#  plus the wave rotation of the j-side sums (6 DPP moves per step of 4 pairs)
#  and an address add per step = 23.75, one 1/sqrt
LOOP_VALU_PER_PAIR = {0: 18.0, 1: 23.75}
LOOP_PAIRS_PER_ITEM = {0: 1, 1: 2}      # directed pairs per loop item (a mutual item serves both bodies)
KERNEL_NAME = {0: "k_force (pairwise FP64 pair loop)", 1: "k_force_mut (mutual FP64 pair loop)"}
BATCH_T_END = 1e-2
BATCH_ETA = 1e-12
# HBM bytes per k_force launch on this workload, from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on a plain 256 MiB copy;
# valid only for the force-kernel and launch-planning sources with this hash.
# (per force kernel kind; None where not measured for the current sources)
FORCE_TRAFFIC = {
    1: {"sha256": "30b68adc528fefe9ff9616e572258658a064733c094713bbb2d76051faa74e56",
        "fetch_bytes": 6248.03 * 1024 * 2.000, "write_bytes": 29412.10 * 1024 * 1.000,
        # executed FP64 flops (ADD + MUL + 2 FMA + TRANS) per directed pair
        "exec_flops_per_pair": 35.0 / 2},
}


def _force_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels_force.hip", "pair.h", "common.h", "api.hip"):   # api.hip: the launch shapes
        with open(os.path.join(ROOT, "paper_2001_03180_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def force_traffic(kind):
    """Measured HBM bytes per force launch if the kernel is the one measured, else None."""
    t = FORCE_TRAFFIC.get(kind)
    if not t or t["sha256"] != _force_sources_hash():
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def force_exec_flops_per_pair(kind):
    """Executed FP64 flops per directed pair if the kernel is the one measured, else None."""
    return FORCE_TRAFFIC[kind]["exec_flops_per_pair"] if force_traffic(kind) is not None else None


def cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(m, x, v, eta, threads):
    """Oracle on the host (bounded samples): one GBS step on all threads, and
    one force evaluation on one thread."""
    import numpy as np
    import oracle
    p = oracle.params(eta=eta, nthreads=threads)
    parent, X, V, scal = oracle.build_state(m, x, v)
    rho = oracle.deconstruct(parent, X)
    _, _, U, _, _ = oracle.force(m, parent, X, rho, p)
    vt = v - (m[:, None] * v).sum(0) / m.sum()
    scal[1] = U - 0.5 * (m * (vt ** 2).sum(1)).sum()
    H = 1e-5
    t0 = time.perf_counter()
    out = oracle.gbs_step(m, parent, X, V, scal, H, p)
    dt = time.perf_counter() - t0
    n = len(m)
    pairs = out[6] * n * (n - 1)
    t0 = time.perf_counter()
    oracle.force(m, parent, X, rho, oracle.params(eta=eta, nthreads=1))
    dt1 = time.perf_counter() - t0
    return dict(value=pairs / dt, unit="pair-interactions/s", cores=threads, kind="oracle",
                sample=f"one GBS step (k_fix=8: {out[6]} force evaluations) at N_p={n}, "
                       f"{dt:.1f} s on {threads} OpenMP threads; one force evaluation on 1 thread in {dt1:.2f} s",
                one_thread={"value": n * (n - 1) / dt1, "unit": "pair-interactions/s", "cores": 1,
                            "sample": f"one force evaluation at N_p={n}"},
                gbs_steps_per_s=1.0 / dt, cpu_model=cpu_model(), nproc=os.cpu_count())


def bench_batch(M, ctx, threads, do_cpu, n_single=12, n_cpu=32):
    """Batched small systems: systems/s of one launch vs the per-system loop."""
    import concurrent.futures as cf
    import numpy as np
    import torch
    import ics
    off, m, x, v = ics.batch_subsystems()
    sizes = np.diff(off)
    n_sys = len(sizes)
    p = M.params(eta=BATCH_ETA)
    res = {
        "workload": "4096 systems, N_p uniform in 3..64 (central mass 1 + stars 1e-5, radii log-uniform "
                    "[1e-3, 1]; 10% hierarchical triples), seed 401; eta=1e-12, k_fix=8, t_end=1e-2",
        "n_sys": int(n_sys), "n_bodies": int(off[-1]), "t_end": BATCH_T_END, "eta": BATCH_ETA,
    }
    t0 = time.perf_counter()
    # tuning horizon: a third of the run; shorter horizons favour the
    # several-systems-per-wave tiles, whose waves wait for their slowest
    # system more as the systems' step counts drift apart over time
    best = ctx.batch_autotune(off, m, x, v, BATCH_T_END / 3, p=p)
    res["autotune_s"] = time.perf_counter() - t0
    res["launch_shape"] = best
    print(f"[bench] batch autotune: {best}", file=sys.stderr, flush=True)
    dm = torch.tensor(m, device="cuda")
    dx = torch.tensor(x, device="cuda")
    dv = torch.tensor(v, device="cuda")
    ctx.integrate_batch(off, dm, dx, dv, BATCH_T_END, p=p)       # warm-up: graph capture
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xg, vg, st = ctx.integrate_batch(off, dm, dx, dv, BATCH_T_END, p=p)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, kern_ms, pairs = ctx.profile_read()
    ctx.profile_enable(False)
    t0 = time.perf_counter()
    ctx.integrate_batch(off, m, x, v, BATCH_T_END, p=p)          # host arrays: with H2D / D2H
    wall_host = time.perf_counter() - t0
    res.update({
        "systems_per_s": n_sys / wall,
        "wall_s": wall,
        "systems_per_s_with_host_copies": n_sys / wall_host,
        "kernel_ms": kern_ms,
        "pair_interactions_per_s": pairs / (kern_ms * 1e-3),
        "status_ok": int((st["status"] == M.OK).sum()),
        "steps_accepted": int(st["steps_accepted"].sum()),
        "steps_rejected": int(st["steps_rejected"].sum()),
        "force_evals": int(st["force_evals"].sum()),
    })
    print(f"[bench] batch: {n_sys} systems in {wall:.3f} s", file=sys.stderr, flush=True)
    # per-system loop of the same library on a seeded random sample
    rng = np.random.default_rng(7)
    pick = sorted(rng.choice(n_sys, n_single, replace=False).tolist())
    t_single = 0.0
    for s in pick:
        o, e = int(off[s]), int(off[s + 1])
        t0 = time.perf_counter()
        ctx.integrate(m[o:e], x[o:e], v[o:e], 0.0, BATCH_T_END, p)
        t_single += time.perf_counter() - t0
    per_sys = n_single / t_single
    res["per_system_loop"] = {
        "systems_per_s": per_sys,
        "sample": f"{n_single} random systems (seed 7, N_p {[int(sizes[s]) for s in pick]}) integrated one "
                  f"per mstar_integrate call in {t_single:.1f} s",
    }
    res["speedup_vs_per_system"] = res["systems_per_s"] / per_sys
    print(f"[bench] per-system loop: {per_sys:.2f} systems/s", file=sys.stderr, flush=True)
    if do_cpu:
        import oracle
        pick = sorted(np.random.default_rng(11).choice(n_sys, n_cpu, replace=False).tolist())
        po = oracle.params(eta=BATCH_ETA, nthreads=1)

        def one(s):
            o, e = int(off[s]), int(off[s + 1])
            oracle.integrate(m[o:e], x[o:e], v[o:e], 0.0, BATCH_T_END, po)

        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, pick))
        dt = time.perf_counter() - t0
        res["cpu_oracle"] = {
            "systems_per_s": n_cpu / dt, "cores": threads, "kind": "oracle",
            "sample": f"{n_cpu} random systems (seed 11), one per host thread, {dt:.1f} s",
        }
    return res


def bench_adjoint(M, ctx, steps=1000, checkpoint_every=50):
    """Cost of one gradient (adjoint pass) against the forward integration."""
    import numpy as np
    import ics
    m, x, v, _ = ics.workload("plummer256_bh")
    n = len(m)
    p = M.params(eta=1e-12)
    ctx.integrate_record(m, x, v, 0.0, 1e9, 20, p)                  # warm-up
    t0 = time.perf_counter()
    xs, vs, rc, st, H = ctx.integrate_record(m, x, v, 0.0, 1e9, steps, p)
    t_fwd = time.perf_counter() - t0
    seed = np.zeros((n, 3))
    seed[n - 1, 0] = 1.0
    t0 = time.perf_counter()
    gx, gv = ctx.replay_adjoint(m, x, v, 0.0, H, seed, np.zeros((n, 3)), 0.0, checkpoint_every)
    t_adj = time.perf_counter() - t0
    t0 = time.perf_counter()
    ctx.replay(m, x, v, 0.0, H)
    t_rep = time.perf_counter() - t0
    # one call that records and reverses: the integrator feeds each accepted
    # step to the adjoint's forward pass, which runs alongside it
    t0 = time.perf_counter()
    cx, cv, _, _ = ctx.integrate_adjoint(m, x, v, 0.0, 1e9, steps, seed, np.zeros((n, 3)), 0.0, checkpoint_every,
                                         p=p, with_mass=False)
    t_one = time.perf_counter() - t0
    same = bool(np.array_equal(cx, gx) and np.array_equal(cv, gv))
    kf = 8
    ops = 2 * kf * (kf + 1) + kf
    step_bytes = (32 * n * ops + 64 * ops + 255) // 256 * 256   # kept substep states of one step
    store = 2 * min(checkpoint_every, (4 << 30) // (2 * step_bytes)) * step_bytes   # two blocks of steps
    dev_bytes = 32 * n * (2 * ((steps + checkpoint_every - 1) // checkpoint_every) + 2 * checkpoint_every +
                          2 + 4 * kf + 4) + store
    return {
        "workload": "plummer256_bh: Plummer N=256 (seed 501) + central mass 0.01 (N_p=257); eta=1e-12, "
                    f"{steps} accepted GBS steps; gradient of the central mass's end x-position w.r.t. all 6N "
                    "initial coordinates",
        "steps": steps, "rejected_steps": st["steps_rejected"], "t_reached": st["t_reached"],
        "forward_s": t_fwd, "adjoint_s": t_adj, "replay_s": t_rep,
        "fwd_plus_bwd_over_fwd": (t_fwd + t_adj) / t_fwd,
        "integrate_adjoint_s": t_one, "integrate_adjoint_over_fwd": t_one / t_fwd,
        "integrate_adjoint_equals_record_then_adjoint": same,
        "checkpoint_every": checkpoint_every, "adjoint_device_bytes": dev_bytes,
        "grad_norm": float(np.sqrt(np.sum(gx * gx) + np.sum(gv * gv))),
    }


def bench_rebuild(M, ctx, n_cycles=100000, seeds=10, n=379):
    """Coordinate round trips of Sec. 3.5: `seeds` equal-mass Hernquist clusters
    of N = 379, each with the MST and with the chain, n_cycles build /
    deconstruct cycles in one call per stretch (all systems side by side),
    once with compensated centre-of-mass sums and once with plain ones (the
    paper's test; kinds 2 and 3); the energy error of every system after each
    stretch."""
    import math
    import numpy as np
    import ics
    sys_ = [ics.hernquist(n, seed) for seed in range(1, seeds + 1)]
    off = np.cumsum([0] + [n] * (4 * seeds))
    m = np.concatenate([s[0] for s in sys_] * 4)
    x = np.concatenate([s[1] for s in sys_] * 4)
    v = np.concatenate([s[2] for s in sys_] * 4)
    kinds = [0] * seeds + [1] * seeds + [2] * seeds + [3] * seeds

    def energy(s, xx, vv):
        """E = T - U with every term summed exactly rounded (math.fsum)."""
        o, e = off[s], off[s + 1]
        ms, xs_, vs_ = m[o:e], xx[o:e], vv[o:e]
        terms = list(0.5 * ms * (vs_ * vs_).sum(1))
        for i in range(len(ms) - 1):
            d = xs_[i + 1:] - xs_[i]
            terms.extend(-(ms[i] * ms[i + 1:]) / np.sqrt((d * d).sum(1)))
        return math.fsum(terms)

    E0 = [energy(s, x, v) for s in range(4 * seeds)]
    marks = [c for c in (300, 1000, 3000, 10000, 30000, 100000) if c < n_cycles] + [n_cycles]
    curve, done, gpu_s, levels = [], 0, 0.0, None
    xc, vc = x.copy(), v.copy()
    for c in marks:
        t0 = time.perf_counter()
        xs, vs, ml = ctx.rebuild_cycles(off, kinds, m, xc, vc, c - done, 1)
        gpu_s += time.perf_counter() - t0
        xc, vc, done = xs[0].copy(), vs[0].copy(), c
        levels = ml if levels is None else levels
        err = [abs(energy(s, xc, vc) - E0[s]) / abs(E0[s]) for s in range(4 * seeds)]
        q = lambda k: err[k * seeds:(k + 1) * seeds]
        curve.append({"cycles": c, "mst_mean": float(np.mean(q(0))), "mst_sd": float(np.std(q(0))),
                      "chain_mean": float(np.mean(q(1))), "chain_sd": float(np.std(q(1))),
                      "plain_mst_mean": float(np.mean(q(2))), "plain_mst_sd": float(np.std(q(2))),
                      "plain_chain_mean": float(np.mean(q(3))), "plain_chain_sd": float(np.std(q(3)))})
        print(f"[bench] rebuild {c} cycles: compensated sums MST |dE/E| {curve[-1]['mst_mean']:.3e}, chain "
              f"{curve[-1]['chain_mean']:.3e}; plain sums MST {curve[-1]['plain_mst_mean']:.3e}, chain "
              f"{curve[-1]['plain_chain_mean']:.3e} ({gpu_s:.1f} s)", file=sys.stderr, flush=True)
    # CPU baseline: the oracle on a bounded sample, one system, both structures, 200 cycles
    import oracle as orc
    t0 = time.perf_counter()
    for kind in (0, 1):
        orc.rebuild_cycles(sys_[0][0], sys_[0][1], sys_[0][2], kind, 200, 0)
    cpu_s = time.perf_counter() - t0
    return {
        "workload": f"{seeds} equal-mass Hernquist clusters, N={n}, r_half=1 (seeds 1..{seeds}), each with the "
                    f"MST and with the chain, with compensated and with plain centre-of-mass sums; {n_cycles} "
                    "build/deconstruct cycles",
        "mean_level_mst": float(np.mean(levels[:seeds])), "mean_level_chain": float(np.mean(levels[seeds:2 * seeds])),
        "curve": curve,
        "gpu_s": gpu_s,
        "round_trips_per_s": 4 * seeds * n_cycles / gpu_s,
        "cpu_oracle": {"round_trips_per_s": 400 / cpu_s, "cores": 1, "kind": "oracle",
                       "sample": "one cluster, MST and chain, 200 cycles each"},
    }


def _energy(m, x, v, block=1024):
    """E = T - U of a Cartesian state (G = 1), plain numpy in row blocks."""
    import numpy as np
    e = 0.5 * float(np.sum(m * (v * v).sum(1)))
    for i0 in range(0, len(m), block):
        d = x[None, :, :] - x[i0:i0 + block, None, :]
        r = np.sqrt((d * d).sum(2))
        r[np.arange(r.shape[0]), np.arange(i0, i0 + r.shape[0])] = np.inf
        e -= 0.5 * float(np.sum(m[i0:i0 + block, None] * m[None, :] / r))
    return e


def steady_attempts(M, ctx, name, steps, warmup):
    """Pair interactions/s of whole GBS step attempts on a named workload, timed
    like the headline: warm up into the step controller's steady state (the
    first-step halvings over), then `steps` attempts with inputs in HBM."""
    import torch
    import ics
    m, x, v, wl = ics.workload(name)
    n = len(m)
    base = dict(eta=wl["eta"], k_fix=8, n_d=2)
    allow = (M.OK, M.W_TIME_TOL, M.E_MAXSTEPS)
    xw, vw, t1, h1 = x, v, 0.0, 0.0
    att_w = acc_w = 0
    chunk = max(warmup, 1)
    for _ in range(100):
        xw, vw, rc, stw = ctx.integrate(m, xw, vw, t1, wl["t_end"], M.params(max_steps=chunk, h_init=h1, **base),
                                        allow=allow)
        att = stw["steps_accepted"] + stw["steps_rejected"]
        att_w += att
        acc_w += stw["steps_accepted"]
        t1, h1 = stw["t_reached"], stw["h_next"]
        if att_w >= warmup and stw["steps_accepted"] >= 0.8 * att and acc_w >= 10:
            break
        chunk = 10
    mt, xt, vt = (torch.tensor(a, device="cuda") for a in (m, xw, vw))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, rc, st = ctx.integrate(mt, xt, vt, t1, wl["t_end"], M.params(max_steps=steps, h_init=h1, **base),
                                 allow=allow)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    done = st["steps_accepted"] + st["steps_rejected"]
    return {"n_bodies": n, "eta": wl["eta"], "pair_interactions_per_s": st["force_evals"] * n * (n - 1) / wall,
            "ms_per_attempt": wall * 1e3 / max(done, 1), "steps_accepted": st["steps_accepted"],
            "steps_rejected": st["steps_rejected"], "t_start": t1, "warmup_attempts": att_w}


def bench_configs(M, ctx, steps=30, warmup=20):
    """The other single-system configurations: 32-body Plummer (eta 1e-12),
    1000-body Plummer with a central mass (eta 1e-13), 10000-body Plummer with
    a hard binary (eta 1e-13)."""
    out = {}
    for name in ("plummer32", "plummer1000_bh", "plummer10000_binary"):
        out[name] = steady_attempts(M, ctx, name, steps, warmup)
        print(f"[bench] {name}: {out[name]['pair_interactions_per_s']:.3e} pairs/s, "
              f"{out[name]['ms_per_attempt']:.3f} ms per attempt", file=sys.stderr, flush=True)
    return out


def bench_mst(M, ctx, names=("plummer5000_binary", "plummer10000_binary"), steps=20, builds=10):
    """Exact (Sec. 3.2) against divide-and-conquer (Sec. 3.3) spanning trees:
    the tree builders alone on the warmed-up state (device arrays, `builds`
    calls each), the tree length, and `steps` GBS step attempts from the same
    warmed-up state with each builder (a rebuild before every attempt after
    an accepted step, as in the headline measurement)."""
    import numpy as np
    import torch
    import ics
    out = {}
    allow = (M.OK, M.W_TIME_TOL, M.E_MAXSTEPS)
    for name in names:
        m, x, v, wl = ics.workload(name)
        base = dict(eta=wl["eta"], k_fix=8, n_d=2)
        xw, vw, t1, h1, att = x, v, 0.0, 0.0, 0
        for _ in range(100):   # steady state, as the headline measurement
            xw, vw, rc, stw = ctx.integrate(m, xw, vw, t1, wl["t_end"], M.params(max_steps=10, h_init=h1, **base),
                                            allow=allow)
            att += stw["steps_accepted"] + stw["steps_rejected"]
            t1, h1 = stw["t_reached"], stw["h_next"]
            if att >= 25 and stw["steps_accepted"] >= 8:
                break
        mt, xt = torch.tensor(m, device="cuda"), torch.tensor(xw, device="cuda")
        res = {"n_bodies": len(m)}
        for kind, dc in (("exact", False), ("dc", True)):
            parent, _, _ = ctx.mst_build(mt, xt, dc=dc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(builds):
                parent, _, _ = ctx.mst_build(mt, xt, dc=dc)
            torch.cuda.synchronize()
            build_ms = (time.perf_counter() - t0) * 1e3 / builds
            pa = parent.cpu().numpy()
            d = xw - xw[np.where(pa >= 0, pa, np.arange(len(pa)))]
            length = float(np.sqrt((d * d).sum(1)).sum())
            p = M.params(max_steps=steps, h_init=h1, **base)
            if dc:
                p.flags |= M.MST_DC
            vt = torch.tensor(vw, device="cuda")
            ctx.integrate(mt, xt, vt, t1, wl["t_end"], p, allow=allow)   # graph capture, untimed
            vt = torch.tensor(vw, device="cuda")
            xs = torch.tensor(xw, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, rc, st = ctx.integrate(mt, xs, vt, t1, wl["t_end"], p, allow=allow)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            att = st["steps_accepted"] + st["steps_rejected"]
            res[kind] = {"build_ms": build_ms, "tree_length": length, "ms_per_attempt": wall * 1e3 / att,
                         "attempts": att, "accepted": st["steps_accepted"], "rebuilds": st["mst_rebuilds"]}
        res["dc_tree_excess"] = res["dc"]["tree_length"] / res["exact"]["tree_length"] - 1.0
        res["dc_step_saving"] = 1.0 - res["dc"]["ms_per_attempt"] / res["exact"]["ms_per_attempt"]
        out[name] = res
        print(f"[bench] mst {name}: build exact {res['exact']['build_ms']:.3f} ms dc {res['dc']['build_ms']:.3f} ms; "
              f"ms/attempt exact {res['exact']['ms_per_attempt']:.3f} dc {res['dc']['ms_per_attempt']:.3f}; "
              f"tree +{res['dc_tree_excess'] * 100:.1f} %", file=sys.stderr, flush=True)
    return out


def bench_timing(M, ctx, sizes=None, seeds=3, eta=1e-6, sweep_n=1129, sweep_etas=None, do_cpu=True):
    """The N-body timing tests of Sec. 5.4 on one GPU: equal-mass Hernquist
    clusters without hard binaries (M = 1e7 Msun, r_half = 10 pc), integrated
    for 0.1 Myr at eta = 1e-6, `seeds` clusters per size; wall-clock seconds
    per simulated Gyr as in the paper's timing figure.  Then the tolerance
    sweep at N = sweep_n (eta from 1e-6 down to 1e-12)."""
    import numpy as np
    import ics
    sizes = sizes or ics.timing_sizes()
    sweep_etas = sweep_etas or [10.0 ** -k for k in range(6, 13)]
    gyr_per_run = 0.1e-3                                   # 0.1 Myr in Gyr
    allow = (M.OK, M.W_TIME_TOL)

    def run(m, x, v, e):
        ctx.integrate(m, x, v, 0.0, ics.TIMING_T_END, M.params(eta=e, max_steps=1),
                      allow=(M.OK, M.W_TIME_TOL, M.E_MAXSTEPS))      # sizes the context's buffers
        t0 = time.perf_counter()
        x1, v1, rc, st = ctx.integrate(m, x, v, 0.0, ics.TIMING_T_END, M.params(eta=e), allow=allow)
        wall = time.perf_counter() - t0
        return wall, st, abs(_energy(m, x1, v1) / _energy(m, x, v) - 1.0)

    rows, clusters = [], {}
    for n in sizes:
        recs = []
        for seed in range(1, seeds + 1):
            m, x, v, _ = ics.timing_cluster(n, seed)
            if n == sweep_n:
                clusters[seed] = (m, x, v)
            recs.append(run(m, x, v, eta))
        wall = np.array([r[0] for r in recs])
        ev = np.array([r[1]["force_evals"] for r in recs], dtype=float)
        rows.append({"n": n, "wall_s": float(wall.mean()), "s_per_gyr": float(wall.mean() / gyr_per_run),
                     "steps_accepted": float(np.mean([r[1]["steps_accepted"] for r in recs])),
                     "steps_rejected": float(np.mean([r[1]["steps_rejected"] for r in recs])),
                     "force_evals": float(ev.mean()),
                     "pairs_per_s": float(np.sum(ev) * n * (n - 1) / np.sum(wall)),
                     "max_abs_dE_over_E": float(max(r[2] for r in recs))})
        print(f"[bench] timing N={n}: {rows[-1]['wall_s']:.3f} s per 0.1 Myr, "
              f"{rows[-1]['steps_accepted']:.0f}+{rows[-1]['steps_rejected']:.0f} steps", file=sys.stderr, flush=True)
    sweep = []
    if sweep_n in [r["n"] for r in rows]:
        for e in sweep_etas:
            recs = [run(*clusters[seed], e) for seed in sorted(clusters)]
            sweep.append({"eta": e, "wall_s": float(np.mean([r[0] for r in recs])),
                          "steps_accepted": float(np.mean([r[1]["steps_accepted"] for r in recs])),
                          "steps_rejected": float(np.mean([r[1]["steps_rejected"] for r in recs])),
                          "max_abs_dE_over_E": float(max(r[2] for r in recs))})
            print(f"[bench] timing N={sweep_n} eta={e:.0e}: {sweep[-1]['wall_s']:.3f} s", file=sys.stderr, flush=True)
        for r in sweep:
            r["wall_over_eta1e-6"] = r["wall_s"] / sweep[0]["wall_s"]
    out = {"workload": f"equal-mass Hernquist clusters without hard binaries, M=1e7 Msun, r_half=10 pc, "
                       f"0.1 Myr ({ics.TIMING_T_END:.4f} N-body units), eta={eta:g}, {seeds} seeds per N",
           "sizes": rows, "eta_sweep": {"n": sweep_n, "runs": sweep}}
    if do_cpu:
        import oracle as orc
        m, x, v, _ = ics.timing_cluster(379, 1)
        t0 = time.perf_counter()
        orc.integrate(m, x, v, 0.0, ics.TIMING_T_END, orc.params(eta=eta))
        cpu = time.perf_counter() - t0
        out["cpu_oracle"] = {"n": 379, "wall_s": cpu, "s_per_gyr": cpu / gyr_per_run, "cores": 1, "kind": "oracle",
                             "sample": "one N=379 cluster (seed 1), 0.1 Myr"}
    return out


def bench_step_control(M, ctx, safety=(0.6, 0.85, 0.9, 0.95, 1.0), etas=(1e-6, 1e-10, 1e-13)):
    """Work of the step-size controller (eq. hnext) against its safety factor
    a_GBS, at three tolerances: force evaluations, wall time, rejections and
    |dE/E| of whole integrations (three N = 1129 and three N = 4833 timing
    clusters over 0.1 Myr; plummer5000_binary to t = 0.02; plummer1000_bh to
    t = 0.2).  Below eta = 1e-11 a_GBS < 0.8 is skipped: the controller then
    aims at eps = eta a_GBS^(2 k_fix - 1), below the rounding floor of the
    error measure, and the steps shrink without end."""
    import ics
    allow = (M.OK, M.W_TIME_TOL)
    cases = []
    for n in (1129, 4833):
        cases.append((f"timing{n}", [ics.timing_cluster(n, s)[:3] for s in (1, 2, 3)], ics.TIMING_T_END))
    for name, te in (("plummer5000_binary", 0.02), ("plummer1000_bh", 0.2)):
        cases.append((name, [ics.workload(name)[:3]], te))
    rows = []
    for name, systems, te in cases:
        e0 = [_energy(m, x, v) for m, x, v in systems]
        for eta in etas:
            for a in safety:
                if eta < 1e-11 and a < 0.8:
                    continue
                wall = 0.0
                acc = rej = fe = 0
                de = 0.0
                for (m, x, v), e in zip(systems, e0):
                    ctx.integrate(m, x, v, 0.0, te, M.params(eta=eta, a_gbs=a, max_steps=1),
                                  allow=allow + (M.E_MAXSTEPS,))      # sizes the context's buffers
                    t0 = time.perf_counter()
                    x1, v1, rc, st = ctx.integrate(m, x, v, 0.0, te, M.params(eta=eta, a_gbs=a), allow=allow)
                    wall += time.perf_counter() - t0
                    acc += st["steps_accepted"]
                    rej += st["steps_rejected"]
                    fe += st["force_evals"]
                    de = max(de, abs(_energy(m, x1, v1) / e - 1.0))
                rows.append({"workload": name, "eta": eta, "a_gbs": a, "wall_s": wall, "steps_accepted": acc,
                             "steps_rejected": rej, "force_evals": fe, "max_abs_dE_over_E": de})
                print(f"[bench] step control {name} eta={eta:.0e} a_gbs={a}: {fe} force evals, "
                      f"{rej}/{acc + rej} rejected, {wall:.3f} s", file=sys.stderr, flush=True)
    return rows


def trace_union(csv_path, pattern):
    """Busy time of the kernels whose name contains `pattern` in a rocprofv3
    kernel trace (the union of their [start, end] intervals), with their
    launch count and mean duration: the same measure as the benchmark's
    kernel time, from the profiler's own timestamps."""
    import csv
    iv = []
    with open(csv_path, newline="") as fh:
        for row in csv.DictReader(fh):
            if pattern in row["Kernel_Name"]:
                iv.append((int(row["Start_Timestamp"]), int(row["End_Timestamp"])))
    iv.sort()
    busy, lo, hi = 0, None, None
    for a, b in iv:
        if hi is None or a > hi:
            if hi is not None:
                busy += hi - lo
            lo, hi = a, b
        else:
            hi = max(hi, b)
    if hi is not None:
        busy += hi - lo
    n = len(iv)
    return {"kernel": pattern, "launches": n, "busy_us_per_launch": busy / 1e3 / max(n, 1),
            "mean_duration_us": sum(b - a for a, b in iv) / 1e3 / max(n, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=25)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched small-systems measurement")
    ap.add_argument("--batch-only", action="store_true", help="only the batched small-systems measurement")
    ap.add_argument("--mst-only", action="store_true",
                    help="only exact vs divide-and-conquer spanning trees (Sec. 3.2 vs 3.3) at N = 5002 and 10002")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint measurement")
    ap.add_argument("--no-configs", action="store_true", help="skip the other single-system configurations")
    ap.add_argument("--configs-only", action="store_true",
                    help="only the other single-system configurations (N_p = 32, 1001, 10002)")
    ap.add_argument("--adjoint-only", action="store_true", help="only the adjoint measurement")
    ap.add_argument("--rebuild-only", action="store_true",
                    help="only the coordinate round-trip experiment (Sec. 3.5; a few minutes)")
    ap.add_argument("--rebuild-cycles", type=int, default=100000)
    ap.add_argument("--timing-only", action="store_true",
                    help="only the cluster timing tests (Sec. 5.4: 20 sizes x 3 seeds, 0.1 Myr, and the eta sweep)")
    ap.add_argument("--timing-max-n", type=int, default=10000)
    ap.add_argument("--trace-union", nargs=2, metavar=("KERNEL_TRACE_CSV", "NAME"),
                    help="busy time per launch of kernels named NAME in a rocprofv3 kernel trace (no GPU)")
    ap.add_argument("--step-control-only", action="store_true",
                    help="only the controller's safety-factor study (eq. hnext; about two minutes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only a plain 256 MiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library "
              "drives one GPU per process and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.trace_union:
        print(json.dumps(trace_union(*args.trace_union)), flush=True)
        return

    import numpy as np
    import torch
    import ics
    import paper_2001_03180_amd as M

    if args.copy_calibration:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": 3}), flush=True)
        return
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    ctx = M.Context(0)
    if args.adjoint_only:
        print(json.dumps({"adjoint": bench_adjoint(M, ctx)}), flush=True)
        return
    if args.rebuild_only:
        print(json.dumps({"rebuild": bench_rebuild(M, ctx, args.rebuild_cycles)}), flush=True)
        return
    if args.timing_only:
        sizes = [k for k in ics.timing_sizes() if k <= args.timing_max_n]
        print(json.dumps({"timing": bench_timing(M, ctx, sizes, do_cpu=not args.no_cpu)}), flush=True)
        return
    if args.mst_only:
        print(json.dumps({"mst": bench_mst(M, ctx)}), flush=True)
        return
    if args.step_control_only:
        print(json.dumps({"step_control": bench_step_control(M, ctx)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch": bench_batch(M, ctx, threads, not args.no_cpu)}), flush=True)
        return
    if args.configs_only:
        print(json.dumps({"configs_other": bench_configs(M, ctx)}), flush=True)
        return
    m, x, v, wl = ics.workload("plummer5000_binary")
    n = len(m)
    eta = wl["eta"]
    base = dict(eta=eta, k_fix=8, n_d=2)

    # warmup from the initial conditions into the step controller's steady
    # state, whatever --warmup asks: at least that many step attempts, then
    # chunks of 10 until one chunk is at least 80% accepted (the first-step
    # halvings are over), continuing with the controller's proposed step
    allow = (M.OK, M.W_TIME_TOL, M.E_MAXSTEPS)
    xw, vw, t1, h1 = x, v, 0.0, 0.0
    warm_att = warm_acc = 0
    chunk = max(args.warmup, 1)
    for _ in range(100):
        xw, vw, rc, stw = ctx.integrate(m, xw, vw, t1, wl["t_end"], M.params(max_steps=chunk, h_init=h1, **base),
                                        allow=allow)
        att = stw["steps_accepted"] + stw["steps_rejected"]
        warm_att += att
        warm_acc += stw["steps_accepted"]
        t1, h1 = stw["t_reached"], stw["h_next"]
        if warm_att >= args.warmup and stw["steps_accepted"] >= 0.8 * att and warm_acc >= 10:
            break
        chunk = 10
    print(f"[bench] warmup: {warm_att} attempts ({warm_acc} accepted) to t={t1:.3e}", file=sys.stderr, flush=True)
    # timed: continue from the warmed-up state with the controller's step
    mt = torch.tensor(m, device="cuda")
    xt = torch.tensor(xw, device="cuda")
    vt = torch.tensor(vw, device="cuda")
    p = M.params(max_steps=args.steps, h_init=h1, **base)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xo, vo, rc, st = ctx.integrate(mt, xt, vt, t1, wl["t_end"], p, allow=(M.OK, M.W_TIME_TOL, M.E_MAXSTEPS))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # force-kernel timing: HIP events around every force launch (on the
    # stream it runs on) over a second pass of the same steps; kept out of the
    # timed pass because each event pair adds launch gaps.  The kernel time is
    # the union of the launches' intervals (the sum of their durations for
    # launches on one stream; MSTAR_DIV_CHAINS lets two chains overlap).  The
    # roofline is that of the dominant kernel (the one with the most launch
    # time).
    ctx.profile_enable(True)
    ctx.integrate(mt, xt, vt, t1, wl["t_end"], p, allow=(M.OK, M.W_TIME_TOL, M.E_MAXSTEPS))
    all_launches, all_ms, all_pairs = ctx.profile_read()
    per_kind = {k: ctx.profile_read_kernel(k) for k in (0, 1)}
    ctx.profile_enable(False)
    kind = max(per_kind, key=lambda k: per_kind[k][1])
    launches, kern_ms, kern_pairs = per_kind[kind]
    steps_done = st["steps_accepted"] + st["steps_rejected"]
    pairs = st["force_evals"] * n * (n - 1)
    value = pairs / wall
    avg_launch_s = kern_ms * 1e-3 / max(launches, 1)
    flops_per_launch = FLOPS_PER_PAIR * kern_pairs / max(launches, 1)
    achieved = flops_per_launch / avg_launch_s / 1e12
    # instruction-mix ceiling of the pair loop at the clock the chip sustains
    fma_cyc, rsq_cyc = ctx.issue_rates()
    n_simd = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    mix_cycles = (LOOP_VALU_PER_PAIR[kind] * fma_cyc + rsq_cyc) / LOOP_PAIRS_PER_ITEM[kind]
    ceiling_pairs = n_simd * 2.4e9 * 64 / mix_cycles
    launch_pairs_per_s = kern_pairs / (kern_ms * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": steps_done,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / max(steps_done, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "plummer5000_binary: Plummer N=5000 (seed 301) + point-mass binary 2x0.005, a=1e-3, "
                        "e=0.9 (N_p=5002); eta=1e-13, k_fix=8, N_d=2, LogH; one step = one GBS step attempt",
            "n_bodies": n,
            "force_evals": st["force_evals"],
            "steps_accepted": st["steps_accepted"],
            "steps_rejected": st["steps_rejected"],
            "mst_rebuilds": st["mst_rebuilds"],
            "t_start": t1,
            "t_reached": st["t_reached"],
            "warmup_attempts": warm_att,
            "warmup_accepted": warm_acc,
        },
        "gbs_steps_accepted_per_s": st["steps_accepted"] / wall,
        "gbs_step_attempts_per_s": steps_done / wall,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": force_traffic(kind),
            "kernel": KERNEL_NAME[kind],
            "launches": launches,
            "avg_launch_us": avg_launch_s * 1e6,
            "time_base": "busy time of the kernel (union of its launch intervals, HIP events) per launch",
            "all_force_launches": {"launches": all_launches, "avg_launch_us": all_ms * 1e3 / max(all_launches, 1),
                                   "tflops_algorithmic": FLOPS_PER_PAIR * all_pairs / (all_ms * 1e-3) / 1e12,
                                   "by_kernel": {KERNEL_NAME[k]: {"launches": v[0], "ms": v[1]}
                                                 for k, v in per_kind.items()}},
            "algorithmic_flops_per_pair": FLOPS_PER_PAIR,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "executed": None if force_exec_flops_per_pair(kind) is None else {
                "flops_per_pair": force_exec_flops_per_pair(kind),
                "tflops": force_exec_flops_per_pair(kind) * launch_pairs_per_s / 1e12,
                "frac_of_peak": force_exec_flops_per_pair(kind) * launch_pairs_per_s / 1e12 / PEAK_FP64_TFLOPS,
                "note": "FP64 VALU flops as executed per directed pair, rocprofv3 SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64",
            },
            "issue_ceiling": {
                "fma_cycles_per_wave_op": fma_cyc,
                "rsq_cycles_per_wave_op": rsq_cyc,
                "loop_valu_per_item": LOOP_VALU_PER_PAIR[kind],
                "directed_pairs_per_item": LOOP_PAIRS_PER_ITEM[kind],
                "pairs_per_s": ceiling_pairs,
                "tflops_algorithmic": FLOPS_PER_PAIR * ceiling_pairs / 1e12,
                "frac_of_ceiling": launch_pairs_per_s / ceiling_pairs,
                "note": "cycles at the nominal 2.4 GHz; 4.0 per FMA is the nominal peak",
            },
        },
    }
    if not args.no_batch:
        out["batch"] = bench_batch(M, ctx, threads, not args.no_cpu)
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(M, ctx)
    if not args.no_configs:
        out["configs_other"] = bench_configs(M, ctx)
    ctx.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(m, x, v, eta, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
