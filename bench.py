"""Benchmark: batched subsequence DTW GCUPS on one MI355X.

One step = one pass of the whole alignment path over the 100,000-pair uneven
batch (query lengths log-normal, median 1,500 events; regions 1.2-3.0x the
query; 1-50 candidates per read): device-side planning (routing,
longest-first ordering) plus the DTW kernels, inputs resident in HBM.  The
timed path is the persistent, tuned form; the plain batched form (static
assignment, arrival order) is timed on the same inputs beside it.

Prints one JSON line (see the keys below).  --gpus above 1 is refused: the
library runs on one GPU; pairs are independent, so a multi-GPU run would
split the batch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X datasheet figures (the bench reads the CU count on the device).
CLOCK_HZ = 2.4e9
# The FP32 vector figure, 157.3 TFLOP/s = 256 CU x 2.4 GHz x 128 lane-ops x 2
# (an FMA counts two), means 128 FP32 lane-ops per clock per CU: each SIMD
# issues two 32-lane VALU ops per cycle when they pair (dual issue).  The
# recurrence has no FMA, so its op peak is half the FLOP figure.
LANES_PER_CU = 128
VALU_OPS_PER_CELL = 3          # v_sub_f32, v_min3_f32, v_add_f32 with |x|
FP32_VECTOR_PEAK = 157.3e12    # datasheet FP32 vector FLOP/s (credits FMA and packed math)
FLOPS_PER_CELL = 5             # sub, abs, 2 x min, add


def route_cells(b):
    """Cells per kernel route (same routing as the library's planner)."""
    m = b.r_len.astype(np.int64)
    cells = b.q_len.astype(np.int64) * m
    lo = m <= 2048
    hi = (m > 2048) & (m <= 4096)
    long_ = m > 4096
    return {"lo": int(cells[lo].sum()), "hi": int(cells[hi].sum()), "long": int(cells[long_].sum())}


def cpu_baseline(b, seconds: float):
    """The CPU oracle (double precision, threaded over pairs) on a random
    sample of pairs until about `seconds` of work has run."""
    from oracle import oracle
    rng = np.random.default_rng(12345)
    order = rng.permutation(b.n_pairs)
    threads = len(os.sched_getaffinity(0))
    done_cells = 0
    done_pairs = 0
    t0 = time.perf_counter()
    chunk = 64
    used = threads
    while time.perf_counter() - t0 < seconds and done_pairs < b.n_pairs:
        idx = order[done_pairs:done_pairs + chunk]
        sub = b.subset(idx)
        _, _, used = oracle.dtw_batch_f64(sub.q, sub.q_off, sub.q_len, sub.r, sub.r_off, sub.r_len, threads)
        done_cells += sub.cells
        done_pairs += len(idx)
        chunk = min(chunk * 2, 4096)
    dt = time.perf_counter() - t0
    return {"value": done_cells / dt / 1e9, "unit": "GCUPS", "cores": int(used), "kind": "oracle",
            "sample": f"{done_pairs} random pairs ({done_cells:.3e} cells, {dt:.1f} s), float64 recurrence"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--skip-plain", action="store_true", help="time only the tuned path (for profiling runs)")
    ap.add_argument("--opts", type=str, default="", help="JSON dict of rawalign_opts fields for the tuned path")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (pairs are independent: "
              "a multi-GPU run would split the batch, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_05037_amd import lib, workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    props = torch.cuda.get_device_properties(dev)
    cus = props.multi_processor_count
    valu_peak = cus * LANES_PER_CU * CLOCK_HZ

    b = workloads.config2()
    cells = b.cells
    rc = route_cells(b)
    db = lib.DeviceBatch(b)
    stream = torch.cuda.current_stream()

    extra = json.loads(args.opts) if args.opts else {}
    tuned = lib.make_opts(flags=lib.FLAG_TIMING, **extra)
    plain_opts = lib.make_opts(mode=lib.MODE_PLAIN, flags=lib.FLAG_TIMING)

    def timed(opts, steps, warmup):
        for _ in range(warmup):
            db.run(opts=opts)
        torch.cuda.synchronize()
        kt = {"plan_ms": [], "lo_ms": [], "hi_ms": [], "long_ms": []}
        t0 = time.perf_counter()
        for _ in range(steps):
            db.run(opts=opts)
            t = lib.rawalign_last_timing()   # waits for this step's events
            for k in kt:
                kt[k].append(getattr(t, k))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt / steps, {k: float(np.mean(v)) for k, v in kt.items()}

    step_s, kt = timed(tuned, args.steps, args.warmup)
    gcups = cells / step_s / 1e9
    plain_gcups = plain_s = None
    pkt = {}
    if not args.skip_plain:
        plain_s, pkt = timed(plain_opts, max(2, args.steps // 2), 1)
        plain_gcups = cells / plain_s / 1e9

    # dominant kernel: the route with the largest average duration
    names = {"lo_ms": "lo", "hi_ms": "hi", "long_ms": "long"}
    dom = max(names, key=lambda k: kt[k])
    dom_cells = rc[names[dom]]
    achieved = VALU_OPS_PER_CELL * dom_cells / (kt[dom] / 1e3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": valu_peak / 1e12, "unit": "TOP/s",
                "frac": achieved / valu_peak, "traffic": None,
                "kernel": {"lo_ms": "k_single<1..8>", "hi_ms": "k_single<9..16>", "long_ms": "k_multi"}[dom],
                "kernel_avg_ms": kt[dom], "kernel_cells": dom_cells,
                "ops_per_cell": VALU_OPS_PER_CELL,
                "whole_step_frac": gcups * 1e9 * VALU_OPS_PER_CELL / valu_peak,
                "datasheet_fp32_frac": gcups * 1e9 * FLOPS_PER_CELL / FP32_VECTOR_PEAK}

    out = {
        "metric": "DTW GCUPS (FP32) batched vs plain at 1e-4 score tol; p50/p99 chunk latency",
        "value": gcups,
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "config2_uneven_batch", "pairs": b.n_pairs, "reads": int(len(b.cand_off)),
                   "cells": cells, "route_cells": rc, "device": props.name, "cus": cus,
                   "opts": {k: v for k, v in tuned.as_dict().items()}},
        "plain": None if plain_gcups is None else
        {"value": plain_gcups, "unit": "GCUPS", "ms_per_step": plain_s * 1e3, "kernels_ms": pkt},
        "persistent_over_plain": None if plain_gcups is None else gcups / plain_gcups,
        "kernels_ms": kt,
        "roofline": roofline,
        "serving": None,
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(b, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
