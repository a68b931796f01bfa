"""Throughput of the split-step round-trip map on one MI355X.

Metric: grid points x round trips per second at 1024^2, batched vs plain.
A step is one round trip of every cavity of the workload.  The workload is a
set of 1024^2 cavities whose Fresnel number, pump ratio, T1 and R follow the
batched sweep's parameter draws (F log-uniform in [100, 1000], pump U[1.2, 4],
T1 U[200, 5000], R U[0.8, 0.98]; seeded noise fields, sigma = 1e-3), in the
FP64-table precision form (FP32 field).  "batched" advances all cavities
together (grouped row/column pass launches or a persistent kernel per round
trip, replayed as HIP graphs, launch shape from the autotune cache);
"plain" launches the row and column kernels of each cavity separately.

Prints one JSON line.  Inputs are resident in HBM before timing.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
ROW_BYTES_PER_PT = 24          # row pass: field read+write 16 B, inversion read+write 8 B
COL_BYTES_PER_PT = 16          # column pass: field read+write 16 B
TRIP_BYTES_PER_PT = ROW_BYTES_PER_PT + COL_BYTES_PER_PT
ROUGH_BYTES_PER_PT = 8         # row pass with mirror roughness: exp(i psi) read, complex64
TUNE_CACHE = os.path.join(ROOT, "paper_1410_2855_amd", "tune_cache.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1410_2855_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, pts_per_launch: int):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel
    calibration) from the committed rocprofv3 summary, if it was taken on the
    current kernel sources and workload; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)[kernel]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("points_per_launch") != pts_per_launch:
        return None
    return rec.get("bytes_per_launch")


# rocprofv3 commands whose output --summarize turns into the committed
# summaries under profiles/ (run from /tmp with TMPDIR=/tmp; OUT is a scratch
# output folder, /root/repo the repository); WL is empty for the metric's
# workload, else "--workload NAME "
PROFILE_COMMANDS = {
    "kernel_trace": "rocprofv3 --kernel-trace --stats --output-format csv -d OUT/kt -o kt -- "
                    "python3 /root/repo/bench.py WL--steps 200 --warmup 20 --no-cpu-baseline --no-parity",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/pf -o pf -- "
             "python3 /root/repo/bench.py WL--profile --steps 2 --warmup 1",
    "write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/pw -o pw -- "
             "python3 /root/repo/bench.py WL--profile --steps 2 --warmup 1",
}


def profile_commands(workload_flag: str = ""):
    return {k: v.replace("WL", workload_flag) for k, v in PROFILE_COMMANDS.items()}


PASS_KERNELS = {"row_pass": "lsr::k_pass<1, 0,", "column_pass": "lsr::k_pass<1, 1,"}
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 64 * 1024 * 1024 * 4   # the calibration copy of --profile, each way


def _read_csv(path):
    import csv

    with open(path) as f:
        return list(csv.DictReader(f))


def summarize(out_dir: str, workload: str, cavities: int, grid: int, workload_flag: str = ""):
    """Turn rocprofv3 csv output (OUT/kt, OUT/pf, OUT/pw of PROFILE_COMMANDS)
    into text summaries, and for the metric's workload (no workload flag)
    profiles/traffic.json, which the bench line's roofline reads.

    HBM traffic per launch = FETCH_SIZE * (copy bytes / copy FETCH_SIZE) +
    WRITE_SIZE * (copy bytes / copy WRITE_SIZE): both counters are scaled by
    what they read for the device-to-device copy of COPY_BYTES that
    bench.py --profile issues."""
    import glob as _g

    prof = os.path.join(ROOT, "profiles")
    os.makedirs(prof, exist_ok=True)
    stats = _read_csv(_g.glob(os.path.join(out_dir, "kt", "*kernel_stats.csv"))[0])
    pts = cavities * grid * grid
    counters = {}
    scale = {}
    for tag, cname in (("pf", "FETCH_SIZE"), ("pw", "WRITE_SIZE")):
        rows = _read_csv(_g.glob(os.path.join(out_dir, tag, "*counter_collection.csv"))[0])
        rows = [r for r in rows if r["Counter_Name"] == cname]
        copy = max((r for r in rows if COPY_KERNEL in r["Kernel_Name"]), key=lambda r: float(r["Counter_Value"]))
        scale[cname] = COPY_BYTES / (float(copy["Counter_Value"]) * 1024.0)
        for k, pat in PASS_KERNELS.items():
            v = [float(r["Counter_Value"]) for r in rows if pat in r["Kernel_Name"]]
            counters.setdefault(k, {})[cname] = (sum(v) / len(v), len(v))
    algo = {"row_pass": ROW_BYTES_PER_PT * pts, "column_pass": COL_BYTES_PER_PT * pts}
    src = kernel_source_hash()
    traffic = {}
    cmds = profile_commands(workload_flag)
    lines_all = ["rocprofv3 kernel statistics: %s" % workload, "",
                 "command (from /tmp, TMPDIR=/tmp): " + cmds["kernel_trace"], "",
                 "%-12s %8s %12s %12s %12s  %s" % ("share %", "calls", "avg us", "min us", "max us", "kernel")]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        lines_all.append("%-12.2f %8s %12.2f %12.2f %12.2f  %s" % (
            float(r["Percentage"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, r["Name"][:160]))
    with open(os.path.join(prof, "kernel_stats_%dx%d.txt" % (cavities, grid)), "w") as f:
        f.write("\n".join(lines_all) + "\n")
    for k, pat in PASS_KERNELS.items():
        st = [r for r in stats if pat in r["Name"] and ("Shape<%d," % grid) in r["Name"]]
        if not st:
            continue
        r = max(st, key=lambda r: int(r["Calls"]))
        avg_ms = float(r["AverageNs"]) / 1e6
        fetch_kib, nf = counters[k]["FETCH_SIZE"]
        write_kib, nw = counters[k]["WRITE_SIZE"]
        fb = fetch_kib * 1024 * scale["FETCH_SIZE"]
        wb = write_kib * 1024 * scale["WRITE_SIZE"]
        traffic[k] = {"source_hash": src, "points_per_launch": pts, "bytes_per_launch": round(fb + wb),
                      "fetch_bytes": round(fb), "write_bytes": round(wb), "algorithmic_bytes": algo[k],
                      "avg_launch_ms": avg_ms}
        txt = ["%s: %s" % (k, workload), "",
               "kernel: " + r["Name"], "",
               "kernel trace (%d calls): avg %.2f us, min %.2f us, max %.2f us" % (
                   int(r["Calls"]), avg_ms * 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3),
               "algorithmic bytes per launch: %d (%d B/pt x %d pts) -> %.1f GB/s at the trace average" % (
                   algo[k], algo[k] // pts, pts, algo[k] / (avg_ms * 1e-3) / 1e9),
               "",
               "FETCH_SIZE %.1f KiB/dispatch (%d dispatches), copy-calibrated x%.4f -> %.1f MiB" % (
                   fetch_kib, nf, scale["FETCH_SIZE"], fb / 2 ** 20),
               "WRITE_SIZE %.1f KiB/dispatch (%d dispatches), copy-calibrated x%.4f -> %.1f MiB" % (
                   write_kib, nw, scale["WRITE_SIZE"], wb / 2 ** 20),
               "HBM traffic per launch %.1f MiB = %.3f x algorithmic" % ((fb + wb) / 2 ** 20, (fb + wb) / algo[k]),
               "",
               "commands (from /tmp, TMPDIR=/tmp):"] + ["  " + c for c in cmds.values()] + [
               "kernel source hash: " + src]
        with open(os.path.join(prof, "%s_%dx%d.txt" % (k, cavities, grid)), "w") as f:
            f.write("\n".join(txt) + "\n")
    if not workload_flag:
        with open(os.path.join(prof, "traffic.json"), "w") as f:
            json.dump(traffic, f, indent=1)
    print(json.dumps(traffic, indent=1))


# Cavity counts of the working-set sweep (--cache-sweep): 12.6 MB of state
# (FP32 field and inversion) per 1024^2 cavity, from 12.6 MB to 805 MB.
CACHE_SWEEP_COUNTS = (1, 2, 4, 8, 12, 16, 20, 24, 32, 48, 64)
CACHE_SWEEP_CMD = ("rocprofv3 --kernel-trace --output-format csv -d OUT/kt -o kt -- python3 /root/repo/bench.py "
                   "--cache-sweep")


def bench_cache_sweep(args):
    """The batched 1024^2 map on the first c cavities of the sweep workload,
    c in CACHE_SWEEP_COUNTS (grouped engine, default FFT plan), each pass
    timed by dispatch events over 200 eager trips after about 0.3 s of
    untimed ones.  While the state a pass
    streams fits the Infinity Cache, a pass reads what the previous pass
    left there; beyond it the passes run at the HBM rate.  One JSON line per
    count: pass durations and the algorithmic bytes per second."""
    import torch

    from paper_1410_2855_amd import lsr
    from paper_1410_2855_amd.inputs import initial_state, sweep_1024

    lsr.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    every = sweep_1024(max(CACHE_SWEEP_COUNTS))
    for c in CACHE_SWEEP_COUNTS:
        cavs = every[:c]
        plans = [lsr.Plan(cv, prec=lsr.LSR_PREC_FP64TAB, stream=stream) for cv in cavs]
        st = [p.state(*initial_state(cv), device=dev) for p, cv in zip(plans, cavs)]
        Es, Ns = [x[0] for x in st], [x[1] for x in st]
        b = lsr.lsr_batch_create([p.handle for p in plans])
        lsr.lsr_batch_configure(b, engine=1, graph_k=0, shape=0)
        # about 0.3 s of trips first, so that the clocks have settled under load
        lsr.lsr_batch_roundtrips(b, Es, Ns, max(50, 36000 // c))
        row_ms, col_ms, trip_ms = lsr.lsr_batch_time_kernels(b, Es, Ns, 200)
        torch.cuda.synchronize()
        lsr.lsr_batch_destroy(b)
        for p in plans:
            p.close()
        pts = c * 1024 * 1024
        print(json.dumps({"cavities": c, "state_MB": round(pts * 12 / 1e6, 1),
                          "row_us": round(row_ms * 1e3, 2), "column_us": round(col_ms * 1e3, 2),
                          "row_GBps": round(ROW_BYTES_PER_PT * pts / row_ms / 1e6, 1),
                          "column_GBps": round(COL_BYTES_PER_PT * pts / col_ms / 1e6, 1),
                          "trip_GBps": round(TRIP_BYTES_PER_PT * pts / trip_ms / 1e6, 1)}), flush=True)
        del Es, Ns, st
        torch.cuda.empty_cache()


def summarize_cache(out_dir: str):
    """profiles/cache_sweep_1024.txt from a rocprofv3 kernel trace of
    bench.py --cache-sweep: per cavity count (the launch's task count over
    1024/4 row or column blocks per cavity), the average duration of the
    middle-trip row and column passes and their algorithmic bytes per second."""
    import glob as _g

    rows = _read_csv(_g.glob(os.path.join(out_dir, "kt", "*kernel_trace.csv"))[0])
    acc = {}
    for r in rows:
        for k, pat in PASS_KERNELS.items():
            if pat in r["Kernel_Name"] and "Shape<1024," in r["Kernel_Name"]:
                tasks = int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"])
                d = acc.setdefault((tasks // 256, k), [])
                d.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = ["Working-set sweep of the batched map: the first c cavities of the 1024^2 sweep workload, "
             "FP64-table form, grouped engine; middle-trip passes of the warm-up and the 200 timed eager trips "
             "per count", "",
             "command (from /tmp, TMPDIR=/tmp): " + CACHE_SWEEP_CMD, "",
             "%9s %9s %9s %10s %12s %10s %12s" % ("cavities", "state MB", "launches", "row us", "row GB/s",
                                                 "column us", "column GB/s")]
    for c in sorted({c for c, _ in acc}):
        rw, cl = acc.get((c, "row_pass"), []), acc.get((c, "column_pass"), [])
        if not rw or not cl:
            continue
        pts = c * 1024 * 1024
        ra, ca = sum(rw) / len(rw), sum(cl) / len(cl)
        lines.append("%9d %9.1f %9d %10.2f %12.1f %10.2f %12.1f" % (
            c, pts * 12 / 1e6, len(rw), ra, ROW_BYTES_PER_PT * pts / ra / 1e3, ca, COL_BYTES_PER_PT * pts / ca / 1e3))
    lines += ["", "state MB: FP32 field and inversion, 12 B per point; GB/s: algorithmic bytes (24 B/pt row, "
              "16 B/pt column) over the kernel-trace average", "kernel source hash: " + kernel_source_hash()]
    path = os.path.join(ROOT, "profiles", "cache_sweep_1024.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)


def summarize_single(out_dir: str, workload: str, fft_plan: int):
    """profiles/kernel_stats_<workload>.txt from a rocprofv3 kernel trace of
    bench.py --workload <single...>: the one-cavity row and column kernels
    (k_row, k_col) of its eager calls, and the batch kernels (k_pass) of the
    graph-replayed legs, one leg per batch FFT plan of the size."""
    import glob as _g

    stats = _read_csv(_g.glob(os.path.join(out_dir, "kt", "*kernel_stats.csv"))[0])
    cmd = ("rocprofv3 --kernel-trace --stats --output-format csv -d OUT/kt -o kt -- python3 /root/repo/bench.py "
           "--workload %s --fft-plan %d --steps 200 --warmup 50" % (workload, fft_plan))
    lines = ["rocprofv3 kernel statistics: %s, one-cavity FFT plan %d" % (WORKLOADS[workload], fft_plan), "",
             "command (from /tmp, TMPDIR=/tmp): " + cmd, "",
             "%-12s %8s %12s %12s %12s  %s" % ("share %", "calls", "avg us", "min us", "max us", "kernel")]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append("%-12.2f %8s %12.2f %12.2f %12.2f  %s" % (
            float(r["Percentage"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, r["Name"][:160]))
    lines += ["", "kernel source hash: " + kernel_source_hash()]
    path = os.path.join(ROOT, "profiles", "kernel_stats_%s.txt" % workload)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)


# SQ counter passes (at most 8 SQ counters per rocprofv3 run): WL as above
SQ_PASSES = {
    "sqa": "SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE SQ_WAIT_INST_LDS SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
           "SQ_INSTS_LDS SQ_INSTS_VALU SQ_WAVES GRBM_GUI_ACTIVE",
    "sqb": "SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VMEM "
           "SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_WAVE_CYCLES",
}


def sq_commands(workload_flag: str = ""):
    return {k: "rocprofv3 --pmc %s --output-format csv -d OUT/%s -o %s -- python3 /root/repo/bench.py %s"
               "--profile --steps 2 --warmup 1" % (v, k, k, workload_flag) for k, v in SQ_PASSES.items()}


def summarize_sq(out_dir: str, workload: str, cavities: int, grid: int, workload_flag: str = ""):
    """profiles/sq_counters_<cavities>x<grid>.txt from the rocprofv3 csv output
    of the SQ_PASSES runs under OUT: mean per dispatch of the middle-trip form
    of each pass, and the ratios read from them."""
    import glob as _g

    vals = {}
    for tag in SQ_PASSES:
        files = _g.glob(os.path.join(out_dir, tag, "*counter_collection.csv"))
        if not files:
            continue
        for r in _read_csv(files[0]):
            for k, pat in PASS_KERNELS.items():
                if pat in r["Kernel_Name"] and ("Shape<%d," % grid) in r["Kernel_Name"]:
                    vals.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    cmds = sq_commands(workload_flag)
    txt = ["SQ counters of the row and column passes: %s" % workload, "",
           "commands (from /tmp, TMPDIR=/tmp):"] + ["  " + c for c in cmds.values()] + [
           "values: mean per dispatch of the middle-trip form of each pass (sum over shader engines and XCDs)", ""]
    for k, cs in vals.items():
        m = {c: sum(v) / len(v) for c, v in cs.items()}
        txt.append("%s:" % k)
        for c in sorted(m):
            txt.append("  %-24s %16.0f" % (c, m[c]))
        wc = m.get("SQ_WAVE_CYCLES")
        if wc:
            for c, what in (("SQ_WAIT_INST_LDS", "wave cycles waiting on LDS instructions"),
                            ("SQ_WAIT_ANY", "wave cycles waiting on anything"),
                            ("SQ_WAIT_INST_ANY", "wave cycles waiting for any instruction issue"),
                            ("SQ_ACTIVE_INST_VALU", "wave cycles issuing VALU"),
                            ("SQ_ACTIVE_INST_LDS", "wave cycles issuing LDS"),
                            ("SQ_ACTIVE_INST_VMEM", "wave cycles issuing vector memory")):
                if c in m:
                    txt.append("  share of %-45s %.3f" % (what + ":", m[c] / wc))
        if "SQ_LDS_BANK_CONFLICT" in m and "SQ_LDS_IDX_ACTIVE" in m:
            txt.append("  LDS bank-conflict cycles per conflict-free LDS cycle: %.3f"
                       % (m["SQ_LDS_BANK_CONFLICT"] / max(m["SQ_LDS_IDX_ACTIVE"] - m["SQ_LDS_BANK_CONFLICT"], 1)))
        if "SQ_INSTS_LDS" in m and "SQ_INSTS_VALU" in m:
            txt.append("  VALU instructions per LDS instruction: %.1f" % (m["SQ_INSTS_VALU"] / m["SQ_INSTS_LDS"]))
        if "SQ_WAVES" in m and "SQ_WAVE_CYCLES" in m:
            txt.append("  wave lifetime (cycles): %.0f" % (m["SQ_WAVE_CYCLES"] / m["SQ_WAVES"]))
        txt.append("")
    txt.append("kernel source hash: " + kernel_source_hash())
    path = os.path.join(ROOT, "profiles", "sq_counters_%dx%d.txt" % (cavities, grid))
    with open(path, "w") as f:
        f.write("\n".join(txt) + "\n")
    print("\n".join(txt))


# L2-to-fabric request counters (at most 4 TCC counters per run), the
# independent check of the FETCH_SIZE / WRITE_SIZE calibration
EA_PASSES = {
    "ea_rd": "TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum",
    "ea_wr": "TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum",
}


def ea_commands(workload_flag: str = ""):
    return {k: "rocprofv3 --pmc %s --output-format csv -d OUT/%s -o %s -- python3 /root/repo/bench.py %s"
               "--profile --steps 2 --warmup 1" % (v, k, k, workload_flag) for k, v in EA_PASSES.items()}


def summarize_ea(out_dir: str, workload: str, cavities: int, grid: int, workload_flag: str = ""):
    """profiles/traffic_requests_<cavities>x<grid>.txt: HBM bytes per launch
    from the request counters by size (read: 32, 64 and 128-byte requests;
    write: 64-byte requests and the rest as 32-byte), for the passes and for
    the calibration copy of known size, beside the copy-calibrated
    FETCH_SIZE / WRITE_SIZE figures of profiles/traffic.json."""
    import glob as _g

    pts = cavities * grid * grid
    algo = {"row_pass": ROW_BYTES_PER_PT * pts, "column_pass": COL_BYTES_PER_PT * pts}
    vals = {}
    for tag in EA_PASSES:
        files = _g.glob(os.path.join(out_dir, tag, "*counter_collection.csv"))
        if not files:
            continue
        for r in _read_csv(files[0]):
            name = r["Kernel_Name"]
            keys = [k for k, pat in PASS_KERNELS.items() if pat in name and ("Shape<%d," % grid) in name]
            if COPY_KERNEL in name:
                keys = ["copy"]
            for k in keys:
                vals.setdefault(k, {}).setdefault(r["Counter_Name"].replace("_sum", ""), []).append(
                    float(r["Counter_Value"]))
    cmds = ea_commands(workload_flag)
    txt = ["HBM traffic from the L2-to-fabric request counters: %s" % workload, "",
           "commands (from /tmp, TMPDIR=/tmp):"] + ["  " + c for c in cmds.values()] + [""]
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            cal = json.load(f)
    except (OSError, ValueError):
        cal = {}
    for k in ("copy", "row_pass", "column_pass"):
        if k not in vals:
            continue
        m = {c: (max(v) if k == "copy" else sum(v) / len(v)) for c, v in vals[k].items()}
        r32, r64, r128 = m.get("TCC_EA0_RDREQ_32B", 0), m.get("TCC_EA0_RDREQ_64B", 0), m.get("TCC_EA0_RDREQ_128B", 0)
        rd = 32 * r32 + 64 * r64 + 128 * r128
        w, w64 = m.get("TCC_EA0_WRREQ", 0), m.get("TCC_EA0_WRREQ_64B", 0)
        wr = 64 * w64 + 32 * (w - w64)
        txt.append("%s: read requests %d (32 B %d, 64 B %d, 128 B %d) -> %.1f MiB; write requests %d (64 B %d) "
                   "-> %.1f MiB" % (k, m.get("TCC_EA0_RDREQ", 0), r32, r64, r128, rd / 2 ** 20, w, w64, wr / 2 ** 20))
        if k == "copy":
            txt.append("  the copy moves %.1f MiB each way" % (COPY_BYTES / 2 ** 20))
        else:
            txt.append("  requests: %.3f x algorithmic (%d B)" % ((rd + wr) / algo[k], algo[k]))
            if k in cal and cal[k].get("points_per_launch") == pts:
                txt.append("  copy-calibrated FETCH_SIZE + WRITE_SIZE (profiles/traffic.json): %.3f x algorithmic"
                           % (cal[k]["bytes_per_launch"] / algo[k]))
    txt.append("")
    txt.append("kernel source hash: " + kernel_source_hash())
    path = os.path.join(ROOT, "profiles", "traffic_requests_%dx%d.txt" % (cavities, grid))
    with open(path, "w") as f:
        f.write("\n".join(txt) + "\n")
    print("\n".join(txt))


WORKLOADS = {
    "single256": "one cavity at 256^2, F=100, R=0.9, pump 2x, T1=1000, FP64-table form",
    "single1024": "one cavity at 1024^2, F=300, R=0.95, pump 3x, T1=2000, FP64-table form",
    "single2048": "one cavity at 2048^2, F=1000, R=0.9, pump 4x, T1=500, FP64-table form",
    "sweep1024": "%d cavities at 1024^2 (sweep parameter draws), FP64-table form",
    "sweep512": "512 cavities, N uniform in {256, 384, 512, 768, 1024} (sweep draws), FP64-table form",
    "structured4096": "16 cavities at 4096^2, F=1000, periodic pump (M = 45..89 periods), FP64-table form",
}


LOCAL_STEPS = {"b-euler": 0, "b-exact": 1, "class-a": 2}
ENGINES = {0: "persistent", 1: "grouped", 2: "grouped-pipelined"}


def make_workload(name: str, cavities: int):
    from paper_1410_2855_amd.inputs import plain_256, plain_1024, precision_2048, structured_4096, sweep, sweep_1024

    if name.startswith("single"):
        return [{"single256": plain_256, "single1024": plain_1024, "single2048": precision_2048}[name]()], \
            WORKLOADS[name]

    if name == "sweep1024":
        return sweep_1024(cavities), WORKLOADS[name] % cavities
    if name == "sweep512":
        return sweep(512), WORKLOADS[name]
    return structured_4096(16), WORKLOADS[name]


def _oracle_worker(job):
    """One single-threaded oracle process: `trips` round trips of one cavity.
    Returns (grid points x trips, wall-clock start, wall-clock end)."""
    cav, trips = job
    import oracle
    from paper_1410_2855_amd.inputs import initial_state, oracle_params

    e0, n0 = initial_state(cav)
    p = oracle_params(cav)
    t0 = time.time()
    oracle.run(p, e0, n0, trips)
    return cav.N * cav.N * trips, t0, time.time()


def cpu_baseline(cavs, seconds_target: float = 12.0):
    """The FP64 oracle on the host's cores: one single-threaded oracle process
    per core (at most 16, a GPU's share of the host), each running round trips
    of its own cavity of the workload for about seconds_target.  The rate is
    all grid points x trips over the span from the first start to the last
    end."""
    import multiprocessing as mp

    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    work, t0, t1 = _oracle_worker((cavs[0], 1))
    trips = max(1, int(seconds_target / max(t1 - t0, 1e-3)))
    jobs = [(cavs[i % len(cavs)], trips) for i in range(cores)]
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map_async(_oracle_worker, jobs, chunksize=1).get(timeout=4 * seconds_target + 120)
    span = max(r[2] for r in res) - min(r[1] for r in res)
    return {"value": sum(r[0] for r in res) / span, "unit": "grid-pts*round-trips/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d oracle processes (FP64 C, one thread each), %d round trips each of %d of the "
                      "workload's cavities (%s^2)" % (cores, trips, min(cores, len(cavs)),
                                                      "/".join(str(n) for n in sorted({c.N for c in cavs[:cores]})))}


def oracle_per_size(sizes=(256, 384, 512, 768, 1024, 2048, 4096), target_s: float = 1.5):
    """Single-threaded oracle time per round trip at each grid size: the
    median of three runs of k trips (k sized to about target_s per run; one
    run includes the oracle's table set-up, amortised over its k trips).
    Returns the host description and one record per size."""
    import platform
    import statistics

    import oracle
    from paper_1410_2855_amd.inputs import Cavity, initial_state, oracle_params

    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    host = {"cpu": model or platform.processor(), "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)), "threads_used": 1}
    rows = []
    for N in sizes:
        cav = Cavity(N=N, F=300.0, R=0.9, pump_ratio=2.0, T1=1000.0, index=1)
        e0, n0 = initial_state(cav)
        p = oracle_params(cav)
        t0 = time.perf_counter()
        oracle.run(p, e0, n0, 1)
        one = time.perf_counter() - t0
        k = max(1, int(target_s / max(one, 1e-4)))
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.run(p, e0, n0, k)
            runs.append((time.perf_counter() - t0) / k)
        t = statistics.median(runs)
        rows.append({"N": N, "trips_per_run": k, "ms_per_trip": round(t * 1e3, 3),
                     "grid_pts_round_trips_per_s": N * N / t})
    return {"host": host, "per_size": rows}


# (N, batch FFT plan) pairs with an alternative plan compiled
BATCH_PLANS = {(256, 1), (512, 1), (1024, 1), (1024, 2), (2048, 1), (4096, 1)}


def bench_single(args):
    """One cavity alone: lsr_roundtrips calls of --steps trips (one launch per
    pass, no graph), the median of --reps calls; the one-cavity FFT plan from
    --fft-plan, or the autotuner's choice (-1).  Also the same calls replayed
    from graphs (a batch of one), per batch FFT plan."""
    import torch

    from paper_1410_2855_amd import lsr
    from paper_1410_2855_amd.inputs import initial_state

    lsr.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    (cav,), workload = make_workload(args.workload, 1)
    p = lsr.Plan(cav, prec=lsr.LSR_PREC_FP64TAB, stream=torch.cuda.current_stream())
    if args.fft_plan >= 0:
        lsr.lsr_plan_set_fft_plan(p.handle, args.fft_plan)
    else:
        lsr.lsr_autotune(p.handle, None, TUNE_CACHE)
    e, n = p.state(*initial_state(cav), device=dev)
    p.roundtrips(e, n, args.warmup)
    torch.cuda.synchronize()
    per = []
    for _ in range(args.reps):
        t0 = time.perf_counter()
        p.roundtrips(e, n, args.steps)
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t0) / args.steps)
    t = statistics.median(per)
    row_ms, col_ms = lsr.lsr_time_kernels(p.handle, e, n, 20)
    p.sync()
    # the same cavity replayed from HIP graphs: a batch of one, one graph per
    # call of --steps trips, captured before the timed calls; each batch FFT
    # plan of the size (plan 1 of 256 is the one-cavity plan 1)
    graph = {}
    for shape in (0, 1, 2):
        b = lsr.lsr_batch_create([p.handle])
        cfg = lsr.lsr_batch_configure(b, engine=1, graph_k=args.steps, shape=shape)
        if cfg["shape"] != shape or (shape > 0 and (cav.N, shape) not in BATCH_PLANS):
            lsr.lsr_batch_destroy(b)
            continue
        lsr.lsr_batch_prepare(b, args.steps)
        lsr.lsr_batch_roundtrips(b, [e], [n], args.steps)
        torch.cuda.synchronize()
        g = []
        for _ in range(args.reps):
            t0 = time.perf_counter()
            lsr.lsr_batch_roundtrips(b, [e], [n], args.steps)
            torch.cuda.synchronize()
            g.append((time.perf_counter() - t0) / args.steps)
        lsr.lsr_batch_destroy(b)
        graph["plan%d" % shape] = round(statistics.median(g) * 1e6, 2)
    p.close()
    pts = cav.N * cav.N
    out = {"metric": "grid-pts x round-trips/s, one cavity", "value": pts / t, "unit": "grid-pts*round-trips/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3,
           "us_per_trip": t * 1e6, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "c64", "data": "synthetic",
           "config": {"workload": workload, "grid": [cav.N], "cavities": 1, "mode": "one cavity, one launch per pass",
                      "fft_plan": args.fft_plan if args.fft_plan >= 0 else "autotuned"},
           "timing": {"reps": len(per), "statistic": "median", "ms_per_step_each": [round(x * 1e3, 5) for x in per]},
           "kernels_ms": {"row_pass": round(row_ms, 5), "column_pass": round(col_ms, 5)},
           "graph_us_per_trip": graph,
           "hbm_frac_whole_step": round(pts * TRIP_BYTES_PER_PT / t / 1e9 / HBM_PEAK_GBS, 4)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--reps", type=int, default=7,
                    help="timed calls of --steps round trips each; the reported time is their median")
    ap.add_argument("--cavities", type=int, default=64, help="cavities of the 1024^2 workload")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="sweep1024",
                    help="sweep1024 (default, the metric's configuration): 1024^2 cavities with the sweep's "
                         "parameter draws; sweep512: 512 cavities of N in {256..1024}; structured4096: "
                         "16 cavities at 4096^2 with the periodic pump; single256/1024/2048: one cavity alone")
    ap.add_argument("--local-step", choices=sorted(LOCAL_STEPS), default="b-euler",
                    help="local step of the map (b-euler: Eq. (1); b-exact: the rate equation solved over "
                         "a trip; class-a: the saturable gain of the class-A laser)")
    ap.add_argument("--filter-delta", type=float, default=0.0,
                    help="> 0: the renormalization-group filter of this width, in grid spacings, "
                         "replaces the Fresnel step")
    ap.add_argument("--rough-rms", type=float, default=0.0,
                    help="> 0: every cavity's mirror carries a random roughness phase of this rms (rad), "
                         "4-cell correlation; the row pass then also reads exp(i psi), 8 B per point")
    ap.add_argument("--autotune", action="store_true", help="retune the batch and update the cache")
    ap.add_argument("--shape", type=int, default=-1,
                    help=">= 0: run the batch on this FFT plan (0 default, k alternative plan k) instead of "
                         "the cached one")
    ap.add_argument("--fft-plan", type=int, default=-1,
                    help="single-cavity workloads: one-cavity FFT plan (0 default, 1 eight points per lane; "
                         "-1 the autotuner's choice)")
    ap.add_argument("--engine", type=int, default=-1,
                    help=">= 0: run the batch on this engine instead of the cached one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="short batched run for a profiler, plus a copy kernel of known size")
    ap.add_argument("--summarize", metavar="OUT",
                    help="write profiles/ summaries from rocprofv3 csv output under OUT (no GPU)")
    ap.add_argument("--summarize-ea", metavar="OUT",
                    help="write profiles/traffic_requests_*.txt from the request-counter runs under OUT (no GPU)")
    ap.add_argument("--summarize-sq", metavar="OUT",
                    help="write profiles/sq_counters_*.txt from the SQ counter runs under OUT (no GPU)")
    ap.add_argument("--cache-sweep", action="store_true",
                    help="time the batched 1024^2 passes for growing cavity counts (12.6 MB to 805 MB of "
                         "state), one JSON line per count")
    ap.add_argument("--summarize-cache", metavar="OUT",
                    help="write profiles/cache_sweep_1024.txt from a kernel trace of --cache-sweep under OUT "
                         "(no GPU)")
    ap.add_argument("--oracle-sizes", action="store_true",
                    help="time the single-threaded FP64 oracle per round trip at every grid size "
                         "(host only, no GPU) and print one JSON line")
    args = ap.parse_args()
    if args.oracle_sizes:
        print(json.dumps(oracle_per_size()), flush=True)
        return
    if args.summarize_cache:
        summarize_cache(args.summarize_cache)
        return
    if args.summarize_ea:
        if args.workload == "sweep1024":
            summarize_ea(args.summarize_ea, WORKLOADS["sweep1024"] % args.cavities, args.cavities, 1024)
        elif args.workload == "structured4096":
            summarize_ea(args.summarize_ea, WORKLOADS["structured4096"], 16, 4096, "--workload structured4096 ")
        else:
            sys.exit("--summarize-ea covers the single-size workloads (sweep1024, structured4096)")
        return
    if args.summarize_sq:
        if args.workload == "sweep1024":
            summarize_sq(args.summarize_sq, WORKLOADS["sweep1024"] % args.cavities, args.cavities, 1024)
        elif args.workload == "structured4096":
            summarize_sq(args.summarize_sq, WORKLOADS["structured4096"], 16, 4096, "--workload structured4096 ")
        else:
            sys.exit("--summarize-sq covers the single-size workloads (sweep1024, structured4096)")
        return
    if args.summarize:
        if args.workload == "sweep1024":
            summarize(args.summarize, WORKLOADS["sweep1024"] % args.cavities, args.cavities, 1024)
        elif args.workload == "structured4096":
            summarize(args.summarize, WORKLOADS["structured4096"], 16, 4096, "--workload structured4096 ")
        elif args.workload.startswith("single"):
            summarize_single(args.summarize, args.workload, max(args.fft_plan, 0))
        else:
            sys.exit("--summarize covers the single-size and one-cavity workloads")
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: every cavity of the workload is independent and the "
              "whole set runs on a single MI355X; sharding across GPUs is a design note, not a run",
              file=sys.stderr)
        sys.exit(2)
    os.environ.setdefault("LSR_TUNE_CACHE", TUNE_CACHE)
    if args.workload.startswith("single"):
        bench_single(args)
        return
    if args.cache_sweep:
        bench_cache_sweep(args)
        return

    import numpy as np
    import torch

    from paper_1410_2855_amd import lsr
    from paper_1410_2855_amd.inputs import initial_state

    lsr.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    cavs, workload = make_workload(args.workload, args.cavities)
    model = LOCAL_STEPS[args.local_step]
    if model or args.filter_delta > 0:
        cavs = [c.with_(model=model, filter_delta=args.filter_delta * c.dx) for c in cavs]
        workload += "; local step %s%s" % (args.local_step, ", filter %.3g dx" % args.filter_delta
                                           if args.filter_delta > 0 else "")
    # the counter summaries cover the default map only
    variant = bool(model or args.filter_delta > 0 or args.rough_rms > 0)
    row_bpp = ROW_BYTES_PER_PT
    if args.rough_rms > 0:
        cavs = [c.with_(rough_rms=args.rough_rms) for c in cavs]
        workload += "; mirror roughness %.3g rad rms" % args.rough_rms
        row_bpp += ROUGH_BYTES_PER_PT
    plans, Es, Ns = [], [], []
    for c in cavs:
        p = lsr.Plan(c, prec=lsr.LSR_PREC_FP64TAB, stream=stream)
        e, n = p.state(*initial_state(c), device=dev)
        plans.append(p)
        Es.append(e)
        Ns.append(n)
    torch.cuda.synchronize()
    pts = sum(c.N * c.N for c in cavs)

    def run_plain(k):
        for p, e, n in zip(plans, Es, Ns):
            p.roundtrips(e, n, k)

    batch = lsr.lsr_batch_create([p.handle for p in plans])
    if args.autotune:
        lsr.lsr_autotune(None, batch, TUNE_CACHE)
    cfg = lsr.lsr_batch_configure(batch, engine=args.engine, shape=args.shape)

    def run_batched(k):
        lsr.lsr_batch_roundtrips(batch, Es, Ns, k)

    def timed(fn, steps, warmup, reps=1):
        """Seconds per step: `warmup` untimed steps, then `reps` timed calls of
        exactly `steps` steps each, every one bracketed by device
        synchronisation; the median over the calls."""
        fn(warmup)
        torch.cuda.synchronize()
        per = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn(steps)
            torch.cuda.synchronize()
            per.append((time.perf_counter() - t0) / steps)
        return statistics.median(per), per

    if args.profile:
        # calibration copy of known size for the traffic counters: 256 MiB
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        lsr.lsr_batch_prepare(batch, args.warmup)
        lsr.lsr_batch_prepare(batch, args.steps)
        t, _ = timed(run_batched, args.steps, args.warmup)
        print(json.dumps({"profile": True, "ms_per_step": t * 1e3, "config": cfg,
                          "copy_bytes_each_way": x.numel() * 4}), flush=True)
        return

    # the graphs a call of `warmup` or `steps` trips replays are captured here,
    # before any timing
    lsr.lsr_batch_prepare(batch, args.warmup)
    lsr.lsr_batch_prepare(batch, args.steps)
    t_step, t_reps = timed(run_batched, args.steps, args.warmup, args.reps)
    value = pts / t_step
    # dominant kernel: dispatch-timestamp events on the batch's stream, right
    # after the timed batched run (same clocks and cache state)
    row_ms, col_ms, trip_ms = lsr.lsr_batch_time_kernels(batch, Es, Ns, 50)
    # plain one-launch-per-cavity leg: the same trips per call as the batched
    # leg (at least 20), so the per-call first and last row passes weigh the same
    plain_steps = max(20, args.steps)
    t_plain, t_plain_reps = timed(run_plain, plain_steps, max(1, args.warmup), max(3, min(args.reps, 5)))
    plain_value = pts / t_plain
    if cfg["engine"] >= 1:
        # grouped launches (engine 1, or its software-pipelined form 2): one
        # kernel per pass
        kernels = {"row_pass": (row_ms, row_bpp * pts), "column_pass": (col_ms, COL_BYTES_PER_PT * pts)}
    else:
        kernels = {"round_trip": (row_ms, (row_bpp + COL_BYTES_PER_PT) * pts)}
    dom = max(kernels, key=lambda k: kernels[k][0])
    ms, nbytes = kernels[dom]
    achieved = nbytes / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None if variant else load_traffic(dom, pts),
                "kernel": dom, "launch_ms": round(ms, 5), "algorithmic_bytes_per_launch": nbytes,
                "bytes_per_point": nbytes // pts,
                "other_kernels_ms": {k: round(v[0], 5) for k, v in kernels.items() if k != dom},
                "event_trip_ms": round(trip_ms, 5)}

    out = {
        "metric": "grid-pts x round-trips/s at 1024^2 (batched vs plain)" if args.workload == "sweep1024"
                  else "grid-pts x round-trips/s (batched vs plain)",
        "value": value,
        "unit": "grid-pts*round-trips/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": workload,
                   "grid": sorted({c.N for c in cavs}), "cavities": len(cavs), "mode": "batched",
                   "engine": ENGINES.get(cfg["engine"], "?"), "launch": cfg},
        "timing": {"reps": len(t_reps), "statistic": "median",
                   "ms_per_step_each": [round(x * 1e3, 5) for x in t_reps],
                   "trips_per_call": args.steps},
        "plain": {"value": plain_value, "ms_per_step": t_plain * 1e3, "trips_per_call": plain_steps,
                  "reps": len(t_plain_reps)},
        "speedup_batched_vs_plain": value / plain_value,
        "hbm_frac_whole_step": round(pts * (row_bpp + COL_BYTES_PER_PT) / t_step / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
    }

    if not args.no_parity:
        # error vs the FP64 oracle after 50 batched round trips, cavity 0
        import oracle
        from paper_1410_2855_amd.inputs import oracle_params

        for c, e, n in zip(cavs, Es, Ns):
            e0, n0 = initial_state(c)
            e.copy_(torch.from_numpy(e0).to(dev, torch.complex64))
            n.copy_(torch.from_numpy(n0).to(dev, torch.float32))
        run_batched(50)
        torch.cuda.synchronize()
        eo, no, _ = oracle.run(oracle_params(cavs[0]), *initial_state(cavs[0]), 50)
        eg, ng = Es[0].cpu().numpy(), Ns[0].cpu().numpy()
        out["err_vs_fp64"] = {"trips": 50, "cavity": 0,
                              "rel_l2_E": float(np.linalg.norm(eg - eo) / np.linalg.norm(eo)),
                              "rel_l2_N": float(np.linalg.norm(ng - no) / np.linalg.norm(no)),
                              "tolerance": 1e-5}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cavs)
    for p in plans:
        p.sync()
    lsr.lsr_batch_destroy(batch)
    for p in plans:
        p.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
