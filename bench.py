"""Throughput of the split-step round-trip map on one MI355X.

Metric: grid points x round trips per second at 1024^2, batched vs plain.
A step is one round trip of every cavity of the workload.  The workload is a
set of 1024^2 cavities whose Fresnel number, pump ratio, T1 and R follow the
batched sweep's parameter draws (F log-uniform in [100, 1000], pump U[1.2, 4],
T1 U[200, 5000], R U[0.8, 0.98]; seeded noise fields, sigma = 1e-3), in the
FP64-table precision form.  "batched" advances all cavities together
(persistent kernel per round trip, replayed as a HIP graph); "plain" launches
the row and column kernels of each cavity separately.

Prints one JSON line (rank 0).  Inputs are resident in HBM before timing.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
ROW_BYTES_PER_PT = 24          # row pass: field R+W 16 B, inversion R+W 8 B
COL_BYTES_PER_PT = 16          # column pass: field R+W
TRIP_BYTES_PER_PT = ROW_BYTES_PER_PT + COL_BYTES_PER_PT


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1410_2855_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, pts_per_launch: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)[kernel]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("points_per_launch") != pts_per_launch:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(seconds_target: float = 12.0):
    """The FP64 oracle, single-threaded, on the first cavity of the workload:
    as many 1024^2 round trips as fit in about seconds_target."""
    import numpy as np

    import oracle
    from paper_1410_2855_amd.inputs import initial_state, oracle_params, sweep_1024

    cav = sweep_1024(1)[0]
    e0, n0 = initial_state(cav)
    p = oracle_params(cav)
    t0 = time.perf_counter()
    oracle.run(p, e0, n0, 1)
    one = time.perf_counter() - t0
    trips = max(1, int(seconds_target / max(one, 1e-3)))
    t0 = time.perf_counter()
    oracle.run(p, e0, n0, trips)
    dt = time.perf_counter() - t0
    return {"value": cav.N * cav.N * trips / dt, "unit": "grid-pts*round-trips/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d round trips of one 1024^2 cavity of the workload, single-threaded FP64 C" % trips}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--cavities", type=int, default=64)
    ap.add_argument("--mode", choices=["auto", "plain", "batched"], default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true", help="short run for a profiler: no baseline, no parity")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the round-trip map of a cavity set is measured on a "
              "single MI355X (cavities are independent; see the design notes for sharding)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1410_2855_amd import lsr
    from paper_1410_2855_amd.inputs import initial_state, sweep_1024

    lsr.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    cavs = sweep_1024(args.cavities)
    plans, Es, Ns = [], [], []
    for c in cavs:
        p = lsr.Plan(c, prec=lsr.LSR_PREC_FP64TAB, stream=stream)
        e0, n0 = initial_state(c)
        e, n = p.state(e0, n0, device=dev)
        plans.append(p)
        Es.append(e)
        Ns.append(n)
    torch.cuda.synchronize()
    pts = sum(c.N * c.N for c in cavs)

    def run_plain(k):
        for p, e, n in zip(plans, Es, Ns):
            p.roundtrips(e, n, k)

    batch = None
    mode = args.mode
    if mode in ("auto", "batched"):
        try:
            batch = lsr.lsr_batch_create([p.handle for p in plans])
        except lsr.LsrError:
            if mode == "batched":
                raise
            batch = None
    if batch is None:
        mode = "plain"
    else:
        mode = "batched"

    def run_batched(k):
        lsr.lsr_batch_roundtrips(batch, Es, Ns, k)

    def timed(fn, steps, warmup):
        fn(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(steps)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    # plain path: always measured (it is the comparison)
    plain_warm = max(1, args.warmup // 4) if mode == "batched" else args.warmup
    plain_steps = max(1, args.steps // 4) if mode == "batched" else args.steps
    t_plain = timed(run_plain, plain_steps, plain_warm)
    plain_value = pts / t_plain
    result_mode = "plain"
    t_step, value = t_plain, plain_value
    if mode == "batched":
        t_step = timed(run_batched, args.steps, args.warmup)
        value = pts / t_step
        result_mode = "batched"

    for p in plans:
        p.sync()

    # dominant kernel: live HIP-event timing on the plan's stream
    e, n = Es[0], Ns[0]
    row_ms, col_ms = lsr.lsr_time_kernels(plans[0].handle, e, n, 20)
    n2 = cavs[0].N * cavs[0].N
    kernels = {
        "row_pass": (row_ms, ROW_BYTES_PER_PT * n2, n2),
        "column_pass": (col_ms, COL_BYTES_PER_PT * n2, n2),
    }
    dom = max(kernels, key=lambda k: kernels[k][0])
    ms, nbytes, npts = kernels[dom]
    achieved = nbytes / (ms * 1e-3) / 1e9
    traffic = load_traffic(dom, npts)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "launch_ms": round(ms, 5),
                "algorithmic_bytes_per_launch": nbytes,
                "other_kernels_ms": {k: round(v[0], 5) for k, v in kernels.items() if k != dom}}

    out = {
        "metric": "grid-pts x round-trips/s at 1024^2 (batched vs plain)",
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
        "config": {"workload": "%d cavities at 1024^2, sweep parameter draws, FP64-table form" % len(cavs),
                   "grid": 1024, "cavities": len(cavs), "mode": result_mode,
                   "precision": "fp32 field, fp64-built tables"},
        "plain": {"value": plain_value, "ms_per_step": t_plain * 1e3},
        "hbm_frac_whole_step": round(pts * TRIP_BYTES_PER_PT / t_step / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
    }
    if batch is not None:
        out["speedup_batched_vs_plain"] = value / plain_value
    if not args.no_cpu_baseline and not args.profile:
        out["cpu_baseline"] = cpu_baseline()
    if batch is not None:
        lsr.lsr_batch_destroy(batch)
    for p in plans:
        p.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
