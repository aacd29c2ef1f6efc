"""bench.trace_union: the busy time of a kernel from a rocprofv3 kernel trace,
the union of its launches' [start, end] intervals (CPU only)."""
import csv

import bench


def _trace(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for name, a, b in rows:
            w.writerow(["KERNEL_DISPATCH", name, a, b])


def test_disjoint_launches_sum(tmp_path):
    p = tmp_path / "t.csv"
    _trace(p, [("k_force_mut<4>", 0, 1000), ("k_kick", 1000, 1500), ("k_force_mut<4>", 2000, 4000)])
    r = bench.trace_union(str(p), "k_force_mut")
    assert r["launches"] == 2
    assert r["busy_us_per_launch"] == r["mean_duration_us"] == 1.5   # (1000 + 2000) ns / 2


def test_overlapping_and_nested_launches_count_once(tmp_path):
    p = tmp_path / "t.csv"
    # [0, 1000] and [500, 1500] overlap; [600, 700] is nested; [3000, 3100] is apart
    _trace(p, [("k_force_mut", 500, 1500), ("k_force_mut", 0, 1000), ("k_force_mut", 600, 700),
               ("k_force_mut", 3000, 3100), ("k_drift", 0, 5000)])
    r = bench.trace_union(str(p), "k_force_mut")
    assert r["launches"] == 4
    assert abs(r["busy_us_per_launch"] - (1500 + 100) / 1e3 / 4) < 1e-12
    assert abs(r["mean_duration_us"] - (1000 + 1000 + 100 + 100) / 1e3 / 4) < 1e-12


def test_no_matching_kernel(tmp_path):
    p = tmp_path / "t.csv"
    _trace(p, [("k_kick", 0, 10)])
    r = bench.trace_union(str(p), "k_force_mut")
    assert r["launches"] == 0 and r["busy_us_per_launch"] == 0.0


def test_step_control_study_wiring():
    """bench_step_control against a stand-in context: every workload, tolerance
    and safety factor is run (a_GBS < 0.8 skipped below eta = 1e-11) and the
    counts of each workload's systems are summed."""
    import paper_2001_03180_amd.mstar as M

    class Ctx:
        def __init__(self):
            self.calls = []

        def integrate(self, m, x, v, t0, te, p, allow=()):
            self.calls.append((len(m), p.eta, p.a_gbs, p.max_steps))
            return x, v, 0, {"steps_accepted": 3, "steps_rejected": 1, "force_evals": 72}

    ctx = Ctx()
    rows = bench.bench_step_control(M, ctx, safety=(0.6, 0.9), etas=(1e-6, 1e-13))
    # 4 workloads x (2 safety factors at 1e-6 + 1 at 1e-13)
    assert len(rows) == 12
    by = {(r["workload"], r["eta"], r["a_gbs"]): r for r in rows}
    assert ("timing1129", 1e-13, 0.6) not in by
    r = by[("timing4833", 1e-6, 0.6)]
    assert r["force_evals"] == 3 * 72 and r["steps_accepted"] == 9 and r["steps_rejected"] == 3
    assert by[("plummer5000_binary", 1e-13, 0.9)]["force_evals"] == 72
    assert r["max_abs_dE_over_E"] == 0.0
    # each timed run is preceded by a one-step call that sizes the buffers
    sizing = [c for c in ctx.calls if c[3] == 1]
    assert len(sizing) == len(ctx.calls) // 2
