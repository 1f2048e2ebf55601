"""Benchmark: batched subsequence DTW GCUPS on one MI355X.

One step = one pass of the whole alignment path over the 100,000-pair uneven
batch (query lengths log-normal, median 1,500 events; regions 1.2-3.0x the
query; 1-50 candidates per read): device-side planning (routing,
longest-first ordering) plus the DTW kernels, inputs resident in HBM.  The
timed path is the persistent, tuned form; the plain batched form (static
assignment, arrival order) is timed on the same inputs beside it.  A
serving leg then streams reads at a fixed arrival rate in 400-event chunks
through resident rows and reports the p50/p99 chunk latency.

Prints one JSON line (see the keys below).  --gpus above 1 is refused: the
library runs on one GPU; pairs are independent, so a multi-GPU run would
split the batch by cells, one share per GPU.
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


def route_bytes(b):
    """Algorithmic HBM bytes per route: every pair reads its query and region
    once and writes a score and an end (4n + 4m + 8)."""
    m = b.r_len.astype(np.int64)
    by = 4 * b.q_len.astype(np.int64) + 4 * m + 8
    return {"lo": int(by[m <= 2048].sum()), "hi": int(by[(m > 2048) & (m <= 4096)].sum()),
            "long": int(by[m > 4096].sum())}


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
    # the same recurrence on one core, over the next pairs of the same order, about 3 s
    one_cells, one_pairs, t1 = 0, 0, time.perf_counter()
    while time.perf_counter() - t1 < min(3.0, seconds) and done_pairs + one_pairs < b.n_pairs:
        sub = b.subset(order[done_pairs + one_pairs:done_pairs + one_pairs + 1])
        oracle.dtw_batch_f64(sub.q, sub.q_off, sub.q_len, sub.r, sub.r_off, sub.r_len, 1)
        one_cells += sub.cells
        one_pairs += 1
    dt1 = time.perf_counter() - t1
    return {"value": done_cells / dt / 1e9, "unit": "GCUPS", "cores": int(used), "kind": "oracle",
            "sample": f"{done_pairs} random pairs ({done_cells:.3e} cells, {dt:.1f} s), float64 recurrence",
            "one_core": {"value": one_cells / dt1 / 1e9, "unit": "GCUPS", "cores": 1,
                         "sample": f"{one_pairs} further pairs ({one_cells:.3e} cells, {dt1:.1f} s)"}}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_multi_uneven_batch_traffic.txt")
KERNEL_SOURCES = ["dtw_device.h", "dtw_multi.hip", "internal.h"]


def kernel_source_hash() -> str:
    """sha256 of the sources that define the dominant kernel, with comments
    and blank lines removed (so only code changes invalidate the counters)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2310_05037_amd", "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            line = line.split("//", 1)[0].strip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel calibration),
    or None when the summary is missing or the kernel sources changed since
    the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.split("=", 1) for line in fh.read().splitlines() if "=" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    return float(kv["hbm_bytes_per_launch"])


def copy_calibration(mib: int):
    """A plain copy kernel of known size (reads and writes `mib` MiB), for
    scaling the FETCH_SIZE and WRITE_SIZE counters to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}), flush=True)


def serving_leg(n_reads: int, rate: float, streams: int = 3, slots: int = 3):
    """Read Until serving at a fixed arrival rate, in real time: 400-event
    chunks one second apart, up to 10 chunks and 1-50 candidates per read,
    resident rows in an 8 GiB arena, two ticks in flight, each a captured
    graph in which the three route kernels run on their own streams.  A
    short time-compressed run first warms up the graphs and caches."""
    from paper_2310_05037_amd import lib, serve, workloads
    opts = lib.make_opts(streams=streams)
    warm = workloads.serving_workload(300, rate=rate, seed_index=103)
    serve.serve(warm, arena_bytes=1 << 30, time_scale=0.05, timeout=120, opts=opts, slots=slots)
    wl = workloads.serving_workload(n_reads, rate=rate)
    _, st = serve.serve(wl, arena_bytes=8 << 30, time_scale=1.0, timeout=600, opts=opts, slots=slots)
    keep = ("p50_ms", "p99_ms", "p999_ms", "max_ms", "chunks", "reads", "ticks", "jobs", "mapped", "unmapped",
            "failed", "peak_arena_bytes", "wall_s", "gcups", "chunks_per_s", "worst_ms", "tick_device_ms")
    out = {k: st[k] for k in keep if k in st}
    out.update({"rate_reads_per_s": rate, "chunk_events": wl.chunk, "chunk_period_s": wl.period, "streams": streams, "slots": slots,
                "latency": "decision on host minus the moment the chunk was available"})
    return out


def bnb_leg(lib, b, opts, steps: int = 3, block_rows: int = 512):
    """Mapping with early termination on the same batch with its candidates
    in a synthetic chaining order (the true region first for 90% of reads):
    time per batch, the full-table cells per second it stands for, the
    fraction of pairs dropped, and whether every read's decision equals the
    one taken on all candidates' full scores."""
    import torch
    from paper_2310_05037_amd import workloads
    c = workloads.chain_ordered(b, seed=0)
    db = lib.DeviceBatch(c)
    dev = db.q.device
    n_reads = len(c.cand_off)
    cand_off = torch.from_numpy(c.cand_off).to(dev)
    cand_cnt = torch.from_numpy(c.cand_cnt).to(dev)
    n_events = torch.from_numpy(c.n_events).to(dev)
    row_off_np = np.concatenate([[0], np.cumsum(c.r_len.astype(np.int64))[:-1]]).astype(np.int64)
    rows = torch.empty(int(c.r_len.astype(np.int64).sum()), dtype=torch.float32, device=dev)
    row_off = torch.from_numpy(row_off_np).to(dev)
    outs = [torch.empty(n_reads, dtype=t, device=dev) for t in (torch.int32, torch.float64, torch.uint8)]
    full = [torch.empty(n_reads, dtype=t, device=dev) for t in (torch.int32, torch.float64, torch.uint8)]
    db.run(opts=opts)
    lib.rawalign_decide(db.score, cand_off, cand_cnt, n_events, *full)
    max_query = int(c.q_len.max())

    def once():
        lib.rawalign_map_bnb(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, cand_off, cand_cnt, n_events,
                             rows, row_off, db.score, db.end, *outs, max_query=max_query, block_rows=block_rows,
                             opts=opts)
    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        once()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    same = all(torch.equal(a, f) for a, f in zip(outs, full))
    pruned = int((db.end == -3).sum().item())
    return {"ms_per_batch": dt * 1e3, "equivalent_gcups": c.cells / dt / 1e9, "unit": "GCUPS",
            "pairs_dropped": pruned, "pairs": c.n_pairs, "decisions_equal_full": bool(same),
            "block_rows": block_rows, "order": "synthetic chaining order, true region first for 90% of reads",
            "entry_point": "rawalign_map_bnb"}


def single_read_leg(lib, reps: int = 300):
    """The single-read workload (one read of 1,566 events against 10 regions
    of 895 levels): latency per read with the inputs on the device, and end
    to end: the read's events and pair tables copied from pinned host memory,
    DTW, decision, results copied back to pinned host memory.  The reference
    levels stay resident, as a mapper's index would.  Ten pairs cannot fill
    the GPU, so this is latency, not throughput."""
    import torch
    from paper_2310_05037_amd import workloads
    b = workloads.single_read()
    db = lib.DeviceBatch(b)
    stream = torch.cuda.current_stream()
    dev = db.q.device
    cand_off = torch.zeros(1, dtype=torch.int64, device=dev)
    cand_cnt = torch.full((1,), b.n_pairs, dtype=torch.int32, device=dev)
    n_events = torch.full((1,), int(b.q_len[0]), dtype=torch.int32, device=dev)
    outs = [torch.empty(1, dtype=t, device=dev) for t in (torch.int32, torch.float64, torch.uint8)]
    opts = lib.make_opts()

    def run_device():
        db.run(opts=opts, stream=stream)
        lib.rawalign_decide(db.score, cand_off, cand_cnt, n_events, *outs, stream=stream)
    for _ in range(20):
        run_device()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run_device()
    e1.record(stream)
    torch.cuda.synchronize()
    device_us = e0.elapsed_time(e1) / reps * 1e3
    # end to end from pinned host buffers
    h_q = torch.from_numpy(b.q).pin_memory()
    h_tab = [torch.from_numpy(np.ascontiguousarray(x)).pin_memory() for x in (b.q_off, b.q_len, b.r_off, b.r_len)]
    d_tab = [db.q_off, db.q_len, db.r_off, db.r_len]
    h_out = [torch.empty(b.n_pairs, dtype=torch.float32).pin_memory(),
             torch.empty(b.n_pairs, dtype=torch.int32).pin_memory()] + \
            [torch.empty(1, dtype=t).pin_memory() for t in (torch.int32, torch.float64, torch.uint8)]
    lat = []
    for k in range(reps + 20):
        t0 = time.perf_counter()
        db.q.copy_(h_q, non_blocking=True)
        for d, h in zip(d_tab, h_tab):
            d.copy_(h, non_blocking=True)
        run_device()
        for h, d in zip(h_out, [db.score, db.end] + outs):
            h.copy_(d, non_blocking=True)
        stream.synchronize()
        if k >= 20:
            lat.append((time.perf_counter() - t0) * 1e3)
    lat = np.array(lat)
    return {"device_us_per_read": device_us, "end_to_end_ms_p50": float(np.percentile(lat, 50)),
            "end_to_end_ms_p99": float(np.percentile(lat, 99)), "pairs": b.n_pairs, "cells": b.cells,
            "best_is_true_region": bool(int(h_out[2][0]) == int(b.true_pair[0])), "mapped": bool(int(h_out[4][0])),
            "workload": "single_read_10_pairs", "reps": reps}


def span_leg(lib, db, opts, steps: int = 3):
    """Scores, ends and starts of the same batch (rawalign_dtw_span: the
    forward pass, then the reversed query against each region prefix up to
    its end): time per batch, and the cells of the reverse pass."""
    import torch
    n = db.batch.n_pairs
    start = torch.empty(n, dtype=torch.int32, device=db.q.device)

    def once():
        lib.rawalign_dtw_span(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, db.score, db.end, start,
                              opts=opts)
    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        once()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    end = db.end.cpu().numpy().astype(np.int64)
    st = start.cpu().numpy()
    rev_cells = int(np.dot(db.batch.q_len.astype(np.int64), np.maximum(end + 1, 0)))
    fwd = db.batch.cells
    return {"ms_per_batch": dt * 1e3, "forward_cells": fwd, "reverse_cells": rev_cells,
            "gcups_both_passes": (fwd + rev_cells) / dt / 1e9, "unit": "GCUPS",
            "mean_span_levels": float(np.mean(end - st + 1)), "entry_point": "rawalign_dtw_span"}


def path_leg(lib, b, opts, steps: int = 3):
    """Warping paths (Sec. 2.4) of the true candidate of every read of the
    uneven batch (3,901 pairs, the ones a mapper would report):
    rawalign_dtw_path (forward and reverse passes, direction words, trace
    back) against rawalign_dtw_span alone on the same pairs."""
    import torch
    tp = b.true_pair[b.true_pair >= 0]
    sub = b.subset(tp)
    db = lib.DeviceBatch(sub)
    n = sub.n_pairs
    rows = sub.q_len.astype(np.int64)
    path_off = torch.from_numpy(np.concatenate([[0], np.cumsum(rows)[:-1]]).astype(np.int64)).cuda()
    lo = torch.empty(int(rows.sum()), dtype=torch.int32, device="cuda")
    hi = torch.empty_like(lo)
    start = torch.empty(n, dtype=torch.int32, device="cuda")
    dir_off, words = lib.path_workspace(sub.q_len, sub.r_len)
    dir_off = torch.from_numpy(dir_off).cuda()
    dirs = torch.empty(words, dtype=torch.int64, device="cuda")

    def path():
        lib.rawalign_dtw_path(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, dir_off, dirs, path_off, lo, hi,
                              db.score, db.end, start, opts=opts)

    def span():
        lib.rawalign_dtw_span(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, db.score, db.end, start,
                              opts=opts)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3
    span_ms = timed(span)
    path_ms = timed(path)
    l0 = lo[path_off].cpu().numpy()
    end = db.end.cpu().numpy().astype(np.int64)
    st = start.cpu().numpy().astype(np.int64)
    rec = l0 >= 0
    L = end - st + 1
    stripes = (L + 2047) // 2048
    return {"ms_per_batch": path_ms, "span_only_ms": span_ms, "pairs": n, "paths_recorded": int(rec.sum()),
            "mean_interval_levels": float(np.mean(L[rec])), "max_interval_levels": int(L[rec].max()),
            "direction_bytes": int((rows[rec] * 512 * stripes[rec]).sum()), "workspace_bytes": words * 8,
            "entry_point": "rawalign_dtw_path", "workload": "uneven_batch_true_candidates"}


def banded_leg(lib, valu_peak: float, opts=None, steps: int = 5, warmup: int = 1):
    """Banded DTW (Sec. 2.4.3) of whole chains: the 100,000 chained segments
    of the anchored workload (read events from the first anchor to the last
    against the levels they span, about 3.3 events per level) with a band
    20% of the segment on each side of the diagonal; the same pairs through
    the full-table path beside it."""
    import torch
    from paper_2310_05037_amd import workloads
    ab = workloads.anchored_chains()
    b, band = workloads.chained_segments(ab)
    db = lib.DeviceBatch(b)
    dband = torch.from_numpy(band).to(db.q.device)
    stream = torch.cuda.current_stream()

    def run_band():
        lib.rawalign_dtw_band(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, dband, db.score, db.end,
                              stream=stream)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps
    band_ms = timed(run_band)
    end = db.end.cpu().numpy()
    # the same pairs with bands of 5% and 10% of the segment on each side
    narrow_ms = {}
    for frac in (0.05, 0.10):
        nb = torch.from_numpy(np.ceil(frac * b.r_len).astype(np.int32)).to(db.q.device)
        narrow_ms[frac] = timed(lambda: lib.rawalign_dtw_band(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len,
                                                              nb, db.score, db.end, stream=stream))
    full_ms = timed(lambda: db.run(opts=opts, stream=stream))
    n = b.q_len.astype(np.int64)
    m = b.r_len.astype(np.int64)
    w = np.minimum(band.astype(np.int64), m - 1)
    # band cells: per row i, the columns of [c(i) - w, c(i) + w] inside [0, m),
    # c(i) = floor(i m / n); counted over chunks of pairs to bound host memory
    band_cells = 0
    for lo in range(0, b.n_pairs, 10000):
        nn, mm, ww = n[lo:lo + 10000], m[lo:lo + 10000], w[lo:lo + 10000]
        rows = np.repeat(np.arange(len(nn)), nn)
        i = np.arange(int(nn.sum())) - np.repeat(np.cumsum(nn) - nn, nn)
        c = i * mm[rows] // nn[rows]
        band_cells += int((np.minimum(c + ww[rows], mm[rows] - 1) - np.maximum(c - ww[rows], 0) + 1).sum())
    frame_cells = int(np.dot(n, 128 * ((2 * w + 1 + 127) // 128)))
    ops = VALU_OPS_PER_CELL * band_cells / (band_ms / 1e3)
    return {"ms_per_batch": band_ms, "full_table_ms": full_ms, "pairs": b.n_pairs, "band_cells": band_cells,
            "full_table_cells": b.cells, "frame_cells": frame_cells,
            "band_gcups": band_cells / (band_ms / 1e3) / 1e9, "full_table_gcups": b.cells / (full_ms / 1e3) / 1e9,
            "speedup_over_full_table": full_ms / band_ms, "unsupported_pairs": int((end == -4).sum()),
            "band_10pct_ms": narrow_ms[0.10], "band_10pct_speedup_over_full_table": full_ms / narrow_ms[0.10],
            "band_5pct_ms": narrow_ms[0.05], "band_5pct_speedup_over_full_table": full_ms / narrow_ms[0.05],
            "roofline": {"bound": "alu", "achieved": ops / 1e12, "peak": valu_peak / 1e12, "unit": "TOP/s",
                         "frac": ops / valu_peak, "over": "band cells at 3 VALU each"},
            "entry_point": "rawalign_dtw_band", "workload": "chained_segments_100000"}


def anchored_leg(lib, valu_peak: float, steps: int = 10, warmup: int = 2):
    """Anchor-guided alignment (Sec. 2.4.2) of 100,000 candidate chains of
    reads shaped like the uneven batch: global DTW of every gap between
    anchors (one gap per lane up to 64 levels, striped kernels above), chain
    sums and the per-read decision.  Reports the time per batch, the gap cells
    per second, and the full tables the chains' spans would have needed."""
    import torch
    from paper_2310_05037_amd import workloads
    ab = workloads.anchored_chains()
    da = lib.DeviceAnchored(ab)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        da.run(stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        da.run(stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    dev_ms = ev0.elapsed_time(ev1) / steps
    _, _, best, _, mapped = da.results()
    span_cells = int(np.dot(ab.chain_events.astype(np.int64), ab.chain_levels.astype(np.int64)))
    tiny = ab.gap_r_len <= 64
    ops = VALU_OPS_PER_CELL * ab.cells / (dev_ms / 1e3)
    return {"ms_per_batch": dt * 1e3, "device_ms_per_batch": dev_ms, "chains": ab.n_chains, "gaps": ab.n_gaps,
            "roofline": {"bound": "alu", "achieved": ops / 1e12, "peak": valu_peak / 1e12, "unit": "TOP/s",
                         "frac": ops / valu_peak, "over": "whole call: planning, gap kernels, chain sums, decision"},
            "gaps_one_per_lane": int(tiny.sum()), "gap_cells": ab.cells,
            "gap_gcups": ab.cells / (dev_ms / 1e3) / 1e9, "chains_per_s": ab.n_chains / (dev_ms / 1e3),
            "chain_span_cells": span_cells,
            "true_chain_wins": float((best == ab.true_chain).mean()), "mapped": float(mapped.mean()),
            "entry_points": ["rawalign_dtw_global_batch", "rawalign_chain_decide"],
            "workload": "anchored_chains_100000"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--skip-plain", action="store_true", help="time only the tuned path (for profiling runs)")
    ap.add_argument("--skip-anchored", action="store_true", help="leave out the anchor-guided alignment leg")
    ap.add_argument("--only-path", action="store_true",
                    help="run only the warping-path leg and print its JSON (for profiling runs)")
    ap.add_argument("--only-banded", action="store_true",
                    help="run only the banded-DTW leg and print its JSON (for profiling runs)")
    ap.add_argument("--only-anchored", action="store_true",
                    help="run only the anchor-guided alignment leg and print its JSON (for profiling runs)")
    ap.add_argument("--opts", type=str, default="", help="JSON dict of rawalign_opts fields for the tuned path")
    ap.add_argument("--no-autotune", action="store_true", help="time the library defaults instead of tuned settings")
    ap.add_argument("--serving-reads", type=int, default=20000, help="reads in the serving leg (0: skip it)")
    ap.add_argument("--serving-rate", type=float, default=2000.0)
    ap.add_argument("--serving-slots", type=int, default=3, help="serving ticks in flight")
    ap.add_argument("--serving-streams", type=int, default=3, choices=(1, 3),
                    help="library streams for the serving extension (3: the three route kernels concurrently)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a copy kernel of this size (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (pairs are independent: "
              "a multi-GPU run would split the batch by cells, one share per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_05037_amd import lib, workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    props = torch.cuda.get_device_properties(dev)
    cus = props.multi_processor_count
    valu_peak = cus * LANES_PER_CU * CLOCK_HZ
    if args.only_anchored:
        print(json.dumps({"anchored": anchored_leg(lib, valu_peak, steps=args.steps, warmup=args.warmup)}), flush=True)
        return
    if args.only_path:
        print(json.dumps({"path": path_leg(lib, workloads.uneven_batch(), None, steps=args.steps)}), flush=True)
        return
    if args.only_banded:
        print(json.dumps({"banded": banded_leg(lib, valu_peak, steps=args.steps, warmup=args.warmup)}), flush=True)
        return

    b = workloads.uneven_batch()
    cells = b.cells
    rc = route_cells(b)
    db = lib.DeviceBatch(b)
    stream = torch.cuda.current_stream()

    extra = json.loads(args.opts) if args.opts else {}
    tune_ms = None
    if not args.no_autotune and not extra:
        # The library times its candidate launch settings on this batch and
        # keeps the fastest; the timed path uses it.
        t0 = time.perf_counter()
        best = lib.rawalign_autotune(*db.args())
        tune_ms = (time.perf_counter() - t0) * 1e3
        extra = {k: getattr(best, k) for k in ("mode", "long_kernel", "lo_waves_per_cu", "hi_waves_per_cu",
                                               "long_waves_per_cu", "streams")}
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
    variants = {}
    if not args.skip_plain:
        plain_s, pkt = timed(plain_opts, max(2, args.steps // 2), 1)
        plain_gcups = cells / plain_s / 1e9
        # Same batch with the anti-diagonal kernel for the regions above one
        # stripe (the lane-striped kernels keep the shorter ones).
        ad_opts = lib.make_opts(flags=lib.FLAG_TIMING, long_kernel=lib.LONG_ANTIDIAG)
        ad_s, akt = timed(ad_opts, 2, 1)
        variants["long_antidiag"] = {"value": cells / ad_s / 1e9, "unit": "GCUPS", "ms_per_step": ad_s * 1e3,
                                     "kernels_ms": akt, "long_route_gcups": rc["long"] / akt["long_ms"] / 1e6,
                                     "kernel": "k_antidiag"}

    if not args.skip_plain:
        variants["early_termination"] = bnb_leg(lib, b, lib.make_opts(**extra))
        variants["alignment_start"] = span_leg(lib, db, lib.make_opts(**extra))
        variants["path"] = path_leg(lib, b, lib.make_opts(**extra))
    if not args.skip_anchored:
        variants["anchored"] = anchored_leg(lib, valu_peak)
    if not args.skip_plain:
        variants["single_read"] = single_read_leg(lib)
    if not args.skip_anchored:
        variants["banded"] = banded_leg(lib, valu_peak, lib.make_opts(**extra))

    # dominant kernel: the route with the largest average duration
    names = {"lo_ms": "lo", "hi_ms": "hi", "long_ms": "long"}
    dom = max(names, key=lambda k: kt[k])
    dom_cells = rc[names[dom]]
    achieved = VALU_OPS_PER_CELL * dom_cells / (kt[dom] / 1e3)
    traffic = measured_traffic()
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": valu_peak / 1e12, "unit": "TOP/s",
                "frac": achieved / valu_peak, "traffic": traffic,
                "algorithmic_bytes": route_bytes(b)[names[dom]],
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
        "config": {"workload": "uneven_batch_100000_pairs", "pairs": b.n_pairs, "reads": int(len(b.cand_off)),
                   "cells": cells, "route_cells": rc, "device": props.name, "cus": cus,
                   "opts": {k: v for k, v in tuned.as_dict().items()}, "autotune_ms": tune_ms},
        "plain": None if plain_gcups is None else
        {"value": plain_gcups, "unit": "GCUPS", "ms_per_step": plain_s * 1e3, "kernels_ms": pkt},
        "persistent_over_plain": None if plain_gcups is None else gcups / plain_gcups,
        "kernels_ms": kt,
        "variants": variants,
        "roofline": roofline,
        "serving": None,
        "cpu_baseline": None,
    }
    del db
    torch.cuda.empty_cache()
    if args.serving_reads > 0:
        out["serving"] = serving_leg(args.serving_reads, args.serving_rate, args.serving_streams, args.serving_slots)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(b, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
