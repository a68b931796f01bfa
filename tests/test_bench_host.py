"""Host logic of bench.py, without a GPU: the single-GPU contract, the
rocprofv3 summary that turns counter output into per-launch HBM bytes (both
counters scaled by what they read for a copy of known size), and the rule
that the bench line reports that traffic only for the kernel sources and
workload it was taken on."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


ROW = "void lsr::k_pass<1, 0, 256, 34944, 4, 0, lsr::Shape<1024, 64, 4, 4, 16, 16> >(a, b)"
COL = "void lsr::k_pass<1, 1, 256, 34944, 4, 0, lsr::Shape<1024, 64, 4, 4, 16, 16> >(a, b)"


def _fake_profile(out, copy_fetch_kib, copy_write_kib, row_fetch_kib, row_write_kib, col_fetch_kib, col_write_kib):
    _write_csv(os.path.join(out, "kt", "kt_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs", "Percentage"],
               [[ROW, 100, 30000000, 300000, 290000, 400000, 55.0],
                [COL, 100, 22000000, 220000, 210000, 300000, 40.0],
                [bench.COPY_KERNEL + "(x)", 1, 100000, 100000, 100000, 100000, 5.0]])
    for tag, name, cp, rv, cv in (("pf", "FETCH_SIZE", copy_fetch_kib, row_fetch_kib, col_fetch_kib),
                                  ("pw", "WRITE_SIZE", copy_write_kib, row_write_kib, col_write_kib)):
        _write_csv(os.path.join(out, tag, tag + "_counter_collection.csv"),
                   ["Kernel_Name", "Counter_Name", "Counter_Value"],
                   [[bench.COPY_KERNEL + "(x)", name, cp], [ROW, name, rv], [ROW, name, rv],
                    [COL, name, cv], ["other", name, 1.0]])


def test_summary_scales_each_counter_by_the_copy(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    out = str(tmp_path / "out")
    # the copy moves COPY_BYTES each way; its FETCH_SIZE reads half of them
    # (128-byte requests counted as 64), its WRITE_SIZE all of them
    copy_fetch = bench.COPY_BYTES / 2 / 1024
    copy_write = bench.COPY_BYTES / 1024
    cavities, grid = 2, 1024
    pts = cavities * grid * grid
    row_alg = bench.ROW_BYTES_PER_PT * pts
    # a row pass that reads 12 B/pt and writes 12 B/pt plus 1% more
    row_fetch = row_alg / 2 / 2 / 1024 * 1.01
    row_write = row_alg / 2 / 1024
    col_alg = bench.COL_BYTES_PER_PT * pts
    _fake_profile(out, copy_fetch, copy_write, row_fetch, row_write, col_alg / 2 / 2 / 1024, col_alg / 2 / 1024)
    bench.summarize(out, "test workload", cavities, grid)
    t = json.load(open(tmp_path / "profiles" / "traffic.json"))
    assert t["row_pass"]["points_per_launch"] == pts
    assert t["row_pass"]["algorithmic_bytes"] == row_alg
    # whole bytes
    assert t["row_pass"]["fetch_bytes"] == pytest.approx(row_alg / 2 * 1.01, abs=1)
    assert t["row_pass"]["write_bytes"] == pytest.approx(row_alg / 2, abs=1)
    assert t["column_pass"]["bytes_per_launch"] == pytest.approx(col_alg, abs=1)
    assert t["row_pass"]["avg_launch_ms"] == pytest.approx(0.3)
    assert t["row_pass"]["source_hash"] == bench.kernel_source_hash()
    txt = open(tmp_path / "profiles" / "row_pass_2x1024.txt").read()
    assert "1.005 x algorithmic" in txt
    # the bench line takes the traffic only for the same sources and workload size
    assert bench.load_traffic("row_pass", pts) == t["row_pass"]["bytes_per_launch"]
    assert bench.load_traffic("row_pass", pts // 2) is None
    t["row_pass"]["source_hash"] = "0" * 16
    json.dump(t, open(tmp_path / "profiles" / "traffic.json", "w"))
    assert bench.load_traffic("row_pass", pts) is None
    assert bench.load_traffic("no_such_kernel", pts) is None


def test_cache_sweep_summary_groups_the_passes_by_cavity_count(tmp_path, monkeypatch):
    """The working-set summary takes each middle-trip pass's cavity count
    from its launch size (one task per four-line block, 256 per 1024^2
    cavity) and its bandwidth from the algorithmic bytes."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    out = str(tmp_path / "out")
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Workgroup_Size_X", "Grid_Size_X"]
    rows = []
    t = 0
    for c, row_ns, col_ns in ((2, 10000, 8000), (8, 30000, 20000)):
        for _ in range(3):
            rows.append([ROW, t, t + row_ns, 256, c * 256 * 256])
            rows.append([COL, t, t + col_ns, 256, c * 256 * 256])
            t += 100000
    rows.append([ROW.replace("k_pass<1, 0,", "k_pass<0, 0,"), 0, 5, 256, 2 * 256 * 256])   # a first-trip pass
    _write_csv(os.path.join(out, "kt", "kt_kernel_trace.csv"), hdr, rows)
    bench.summarize_cache(out)
    txt = open(tmp_path / "profiles" / "cache_sweep_1024.txt").read().split("\n")
    table = [l.split() for l in txt if l.strip() and l.split()[0].isdigit()]
    assert [int(r[0]) for r in table] == [2, 8]
    two, eight = table
    assert int(two[2]) == 3 and float(two[3]) == 10.0 and float(two[5]) == 8.0
    pts = 8 * 1024 * 1024
    assert float(eight[4]) == pytest.approx(24 * pts / 30e-6 / 1e9, rel=1e-3)
    assert float(eight[6]) == pytest.approx(16 * pts / 20e-6 / 1e9, rel=1e-3)
    assert "kernel source hash: " + bench.kernel_source_hash() in txt
