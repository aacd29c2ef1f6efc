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
