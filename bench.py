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


EDGE_CAP = 16384   # RAWALIGN_MAX_QUERY_LONG: longer queries keep one stripe up to 4096 levels


def route_masks(b, single_max: int = 4096):
    """Pairs per kernel route, as the library's planner routes them: up to
    2048 levels, up to the single-stripe cut-off (single_max, and up to 4096
    levels for queries too long for a stripe edge column), longer."""
    m = b.r_len.astype(np.int64)
    n = b.q_len.astype(np.int64)
    lo = m <= 2048
    hi = ~lo & ((m <= single_max) | ((m <= 4096) & (n > EDGE_CAP)))
    return {"lo": lo, "hi": hi, "long": ~lo & ~hi}


def route_cells(b, single_max: int = 4096):
    """Cells per kernel route."""
    cells = b.q_len.astype(np.int64) * b.r_len.astype(np.int64)
    return {k: int(cells[v].sum()) for k, v in route_masks(b, single_max).items()}


def route_bytes(b, single_max: int = 4096):
    """Algorithmic HBM bytes per route: every pair reads its query and region
    once and writes a score and an end (4n + 4m + 8)."""
    by = 4 * b.q_len.astype(np.int64) + 4 * b.r_len.astype(np.int64) + 8
    return {k: int(by[v].sum()) for k, v in route_masks(b, single_max).items()}


def stratified_order(b, seed: int = 12345, strata: int = 64):
    """Pairs in an order whose every prefix is spread over the cell-count
    distribution: pairs sorted by cells, cut into `strata` equal groups, one
    random pair from each group in turn."""
    rng = np.random.default_rng(seed)
    cells = b.q_len.astype(np.int64) * b.r_len.astype(np.int64)
    groups = [rng.permutation(g) for g in np.array_split(np.argsort(cells, kind="stable"), strata)]
    order = []
    for k in range(max(len(g) for g in groups)):
        order.extend(int(g[k]) for g in groups if k < len(g))
    return np.array(order, dtype=np.int64)


def cpu_baseline(b, seconds: float, gpu_score=None, gpu_end=None):
    """The CPU oracle (double precision, threaded over pairs) on a sample of
    pairs spread over the cell-count distribution, until about `seconds` of
    work has run.  With the GPU's results of the timed step, the same sample
    also gives their largest relative error against the double oracle and
    the ends that differ from it (score tolerance 1e-4 relative)."""
    from oracle import oracle
    order = stratified_order(b)
    threads = len(os.sched_getaffinity(0))
    done_cells = 0
    done_pairs = 0
    t0 = time.perf_counter()
    chunk = 64
    used = threads
    ref = []
    while time.perf_counter() - t0 < seconds and done_pairs < b.n_pairs:
        idx = order[done_pairs:done_pairs + chunk]
        sub = b.subset(idx)
        s64, e64, used = oracle.dtw_batch_f64(sub.q, sub.q_off, sub.q_len, sub.r, sub.r_off, sub.r_len, threads)
        ref.append((idx, s64, e64))
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
    out = {"value": done_cells / dt / 1e9, "unit": "GCUPS", "cores": int(used), "kind": "oracle",
           "sample": f"{done_pairs} pairs spread over the cell-count distribution ({done_cells:.3e} cells, "
                     f"{dt:.1f} s), float64 recurrence",
           "one_core": {"value": one_cells / dt1 / 1e9, "unit": "GCUPS", "cores": 1,
                        "sample": f"{one_pairs} further pairs ({one_cells:.3e} cells, {dt1:.1f} s)"}}
    if gpu_score is not None and ref:
        idx = np.concatenate([x[0] for x in ref])
        s64 = np.concatenate([x[1] for x in ref])
        e64 = np.concatenate([x[2] for x in ref])
        gs = gpu_score[idx].astype(np.float64)
        rel = np.abs(gs - s64) / np.maximum(np.abs(s64), 1e-30)
        out["parity"] = {"pairs": int(len(idx)), "max_rel_err": float(rel.max()), "tolerance": 1e-4,
                         "within_tolerance": bool((np.abs(gs - s64) <= 1e-4 * np.abs(s64) + 1e-6).all()),
                         "ends_differing_from_f64": int((gpu_end[idx] != e64).sum()),
                         "of": "the timed (tuned, persistent) step's scores and ends"}
    return out


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


PROBE_OPS = ("v_add_f32", "v_sub_f32", "v_min3_f32", "v_max_f32", "dtw_cell(v_sub,v_min3,v_add|x|)")


def valu_rate(iters: int = 20000):
    """Issue rate of VALU instruction forms on this GPU (libvaluprobe.so):
    lane-operations per clock per CU for each form at 4 to 32 resident waves
    per CU, and the shader clock the cycle counter implies.  This is what
    the roofline's op peak (128 FP32 lane-operations per clock per CU, the
    datasheet's 157.3 TFLOP/s without the FMA credit) rests on; and the rate
    of the constant clock behind the pipelined kernels' wait caps."""
    import ctypes
    import torch  # noqa: F401  (loads the HIP runtime first)
    path = os.path.join(ROOT, "paper_2310_05037_amd", "libvaluprobe.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with paper_2310_05037_amd/build.py")
    L = ctypes.CDLL(path)
    d = ctypes.c_double
    L.valu_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(d), ctypes.POINTER(d),
                             ctypes.POINTER(d)]
    out = {"unit": "FP32 lane-operations per clock per CU", "iters": iters, "chains_per_wave": 8, "forms": {}}
    for op, name in enumerate(PROBE_OPS):
        row = {}
        for w in (4, 8, 16, 32):
            rate, ghz, ms = d(), d(), d()
            rc = L.valu_probe(op, w, iters, ctypes.byref(rate), ctypes.byref(ghz), ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError(f"valu_probe({name}, {w}) failed: {rc}")
            row[f"{w}_waves_per_cu"] = {"lane_ops_per_clk_per_cu": rate.value, "clock_ghz": ghz.value,
                                        "kernel_ms": ms.value}
        out["forms"][name] = row
    # Rate of the constant clock the pipelined kernels' capped waits count
    # (s_memrealtime): ticks over one second of host wall time.
    L.clock_probe.argtypes = [ctypes.c_int, ctypes.POINTER(d), ctypes.POINTER(d)]
    ticks, secs = d(), d()
    rc = L.clock_probe(1000, ctypes.byref(ticks), ctypes.byref(secs))
    if rc != 0:
        raise RuntimeError(f"clock_probe failed: {rc}")
    out["memrealtime"] = {"ticks": ticks.value, "seconds": secs.value, "hz": ticks.value / secs.value}
    return out


def serving_leg(n_reads: int, rate: float, streams: int = 3, slots: int = 3, cap_frac: float = 0.5,
                pipe_waves: int = 8, single_max: int = 2048):
    """Read Until serving at a fixed arrival rate, in real time: 400-event
    chunks one second apart, up to 10 chunks and 1-50 candidates per read,
    30% of the reads off target (decoy candidates only: they never map and
    stream every chunk), the decision's match bonus set for this data's noise
    floor (workloads.SYNTHETIC_B_MATCH), resident rows in an 8 GiB arena,
    three ticks in flight, each a captured graph in which the three route
    kernels run on their own streams, regions above `single_max` levels
    shared by `pipe_waves` waves each (the pipelined kernel; 0: one wave per
    pair).  A short time-compressed run first warms up the graphs and
    caches.  The same reads then run again with an
    arena cap of `cap_frac` of the first run's peak: admission waits
    (back-pressure), the cap holds, and every read's per-chunk results must
    equal the first run's."""
    from paper_2310_05037_amd import lib, serve, workloads
    kw = dict(streams=streams, single_max=single_max)
    if pipe_waves:
        kw.update(long_kernel=lib.LONG_PIPELINE, pipe_waves=pipe_waves)
    opts = lib.make_opts(**kw)
    bm = workloads.SYNTHETIC_B_MATCH
    warm = workloads.serving_workload(300, rate=rate, seed_index=103)
    serve.serve(warm, arena_bytes=1 << 30, time_scale=0.05, timeout=120, opts=opts, slots=slots, b_match=bm)
    wl = workloads.serving_workload(n_reads, rate=rate)
    eng, st = serve.serve(wl, arena_bytes=8 << 30, time_scale=1.0, timeout=600, opts=opts, slots=slots,
                          b_match=bm)
    keep = ("p50_ms", "p99_ms", "p999_ms", "max_ms", "chunks", "reads", "chunks_per_read", "max_chunks_per_read",
            "reads_3plus_chunks", "ticks", "jobs", "cells", "mapped", "unmapped", "failed", "peak_arena_bytes",
            "arena_bytes", "peak_queued_reads", "wall_s", "gcups", "chunks_per_s", "worst_ms", "tick_device_ms")
    out = {k: st[k] for k in keep if k in st}
    off = sum(1 for rd in wl.reads if rd.true_cand < 0)
    out.update({"rate_reads_per_s": rate, "chunk_events": wl.chunk, "chunk_period_s": wl.period,
                "streams": streams, "slots": slots, "opts": {k: v for k, v in kw.items()},
                "off_target_reads": off, "b_match": bm,
                "threshold": eng.threshold,
                "latency": "decision on host minus the moment the chunk was available"})
    cap = int(st["peak_arena_bytes"] * cap_frac) // 4 * 4
    eng2, st2 = serve.serve(wl, arena_bytes=cap, time_scale=1.0, timeout=600, opts=opts, slots=slots, b_match=bm)
    same = all(a.status == b.status and len(a.results) == len(b.results) and
               all(x[:3] == y[:3] and np.array_equal(x[3].view(np.uint32), y[3].view(np.uint32)) and
                   np.array_equal(x[4], y[4]) for x, y in zip(a.results, b.results))
               for a, b in zip(eng.reads, eng2.reads))
    out["capped"] = {k: st2[k] for k in ("p50_ms", "p99_ms", "p999_ms", "max_ms", "chunks", "peak_arena_bytes",
                                         "arena_bytes", "peak_queued_reads", "failed", "wall_s") if k in st2}
    out["capped"].update({"cap_fraction_of_uncapped_peak": cap_frac, "results_equal_uncapped": bool(same)})
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
    uneven batch (3,901 pairs, the ones a mapper would report), two ways:
    rawalign_dtw_path alone (forward and reverse passes, direction words,
    trace back) into a workspace sized for the whole region of every pair;
    and rawalign_dtw_span, then rawalign_dtw_path with the span outputs
    given, into a workspace sized from the aligned intervals.  Both must
    give the same paths."""
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
    paths_full = (lo.cpu().numpy(), hi.cpu().numpy())
    end = db.end.cpu().numpy().astype(np.int64)
    st = start.cpu().numpy().astype(np.int64)
    rec = l0 >= 0
    L = end - st + 1
    stripes = (L + 2047) // 2048
    del dirs
    torch.cuda.empty_cache()
    # The span's intervals size the workspace exactly; the path call then
    # skips the span passes.
    x_off, x_words = lib.path_workspace_exact(sub.q_len, end, st)
    x_off = torch.from_numpy(x_off).cuda()
    x_dirs = torch.empty(max(x_words, 1), dtype=torch.int64, device="cuda")
    given = lib.make_opts(**{k: v for k, v in (opts.as_dict() if opts is not None else {}).items() if k != "flags"},
                          flags=lib.FLAG_SPAN_GIVEN)

    def path_given():
        lib.rawalign_dtw_path(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, x_off, x_dirs, path_off, lo, hi,
                              db.score, db.end, start, opts=given)
    given_ms = timed(path_given)
    same = bool(np.array_equal(lo.cpu().numpy(), paths_full[0]) and np.array_equal(hi.cpu().numpy(), paths_full[1]))
    return {"ms_per_batch": path_ms, "span_only_ms": span_ms, "pairs": n, "paths_recorded": int(rec.sum()),
            "mean_interval_levels": float(np.mean(L[rec])), "max_interval_levels": int(L[rec].max()),
            "direction_bytes": int((rows[rec] * 512 * stripes[rec]).sum()), "workspace_bytes": words * 8,
            "exact_workspace_bytes": x_words * 8, "path_after_span_ms": given_ms,
            "exact_workspace_paths_equal": same,
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


def banded_regions_leg(lib, db, full_ms: float, steps: int = 3):
    """Banded DTW of the uneven batch's candidate regions (1.2 to 3 times
    the read) at a band of 20% of the region: time per batch against the
    full table's, and the cells inside the band."""
    import torch
    b = db.batch
    band = np.ceil(0.2 * b.r_len).astype(np.int32)
    dband = torch.from_numpy(band).to(db.q.device)
    stream = torch.cuda.current_stream()

    def run():
        lib.rawalign_dtw_band(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, dband, db.score, db.end,
                              stream=stream)
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    end = db.end.cpu().numpy()
    n = b.q_len.astype(np.int64)
    m = b.r_len.astype(np.int64)
    w = np.minimum(band.astype(np.int64), m - 1)
    band_cells = 0
    for lo in range(0, b.n_pairs, 5000):
        nn, mm, ww = n[lo:lo + 5000], m[lo:lo + 5000], w[lo:lo + 5000]
        rows = np.repeat(np.arange(len(nn)), nn)
        i = np.arange(int(nn.sum())) - np.repeat(np.cumsum(nn) - nn, nn)
        c = i * mm[rows] // nn[rows]
        band_cells += int(np.maximum(np.minimum(c + ww[rows], mm[rows] - 1) - np.maximum(c - ww[rows], 0) + 1,
                                     0).sum())
    return {"ms_per_batch": ms, "full_table_ms": full_ms, "speedup_over_full_table": full_ms / ms,
            "band_cells": band_cells, "full_table_cells": b.cells, "band_gcups": band_cells / (ms / 1e3) / 1e9,
            "unsupported_pairs": int((end == -4).sum()), "pairs": b.n_pairs,
            "entry_point": "rawalign_dtw_band", "workload": "uneven_batch_100000_pairs, band 20% of the region"}


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


def note(msg: str):
    """One progress line on stderr (stdout carries only the result line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def timed_steps(lib, db, opts, steps: int, warmup: int):
    """Seconds per call of rawalign_dtw_batch_ex on a DeviceBatch and the mean
    per-kernel times (HIP events on the streams the kernels run on)."""
    import torch
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


KERNEL_NAMES = {"lo_ms": "k_single<1..8>", "hi_ms": "k_single<9..16>", "long_ms": "k_multi"}


def dominant_roofline(b, kt, valu_peak, long_name="k_multi", single_max: int = 4096):
    """Roofline block of the route kernel with the largest average time."""
    names = {"lo_ms": "lo", "hi_ms": "hi", "long_ms": "long"}
    rc = route_cells(b, single_max)
    dom = max(names, key=lambda k: kt[k])
    achieved = VALU_OPS_PER_CELL * rc[names[dom]] / (kt[dom] / 1e3)
    kernel = dict(KERNEL_NAMES, long_ms=long_name)[dom]
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": valu_peak / 1e12, "unit": "TOP/s",
            "frac": achieved / valu_peak, "kernel": kernel, "kernel_avg_ms": kt[dom],
            "kernel_cells": rc[names[dom]], "algorithmic_bytes": route_bytes(b, single_max)[names[dom]],
            "ops_per_cell": VALU_OPS_PER_CELL}


def batch_config_leg(lib, b, workload, valu_peak, tuned_extra, steps: int, warmup: int, antidiag: bool = False,
                     pipeline: bool = False):
    """One batch workload timed three or four ways on the same inputs: plain
    (static assignment, arrival order), persistent with the library
    defaults, persistent with the tuned settings, and (antidiag) the tuned
    settings with the anti-diagonal kernel for regions above one stripe.
    Every form must return the same bits."""
    import torch
    db = lib.DeviceBatch(b)
    forms = [("plain", dict(mode=lib.MODE_PLAIN)), ("persistent_default", {})]
    if tuned_extra:
        forms.append(("persistent_tuned_on_uneven_batch", tuned_extra))
    if antidiag:
        forms.append(("antidiag", dict(long_kernel=lib.LONG_ANTIDIAG)))
    if pipeline:
        for w in (2, 4, 8):
            forms.append((f"pipeline_{w}_waves", dict(long_kernel=lib.LONG_PIPELINE, pipe_waves=w)))
    # the autotuner on this batch itself
    t0 = time.perf_counter()
    best = lib.rawalign_autotune(*db.args())
    tune_ms = (time.perf_counter() - t0) * 1e3
    self_tuned = {k: v for k, v in best.as_dict().items() if k != "flags"}
    forms.append(("persistent_tuned", self_tuned))
    out = {"workload": workload, "pairs": b.n_pairs, "cells": b.cells, "route_cells": route_cells(b),
           "tuned_opts": self_tuned, "autotune_ms": tune_ms}
    ref = None
    same = True
    for name, kw in forms:
        s, kt = timed_steps(lib, db, lib.make_opts(flags=lib.FLAG_TIMING, **kw), steps, warmup)
        res = db.results()
        if ref is None:
            ref = (res[0].copy(), res[1].copy())
        else:
            same = same and np.array_equal(res[0].view(np.uint32), ref[0].view(np.uint32)) and \
                np.array_equal(res[1], ref[1])
        kind = kw.get("long_kernel", 0)
        out[name] = {"value": b.cells / s / 1e9, "unit": "GCUPS", "ms_per_step": s * 1e3, "kernels_ms": kt,
                     "roofline": dominant_roofline(b, kt, valu_peak,
                                                   {1: "k_antidiag", 2: "k_pipe"}.get(kind, "k_multi"),
                                                   kw.get("single_max") or 4096)}
    out["all_forms_bit_identical"] = bool(same)
    del db
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--skip-plain", action="store_true", help="time only the tuned path (for profiling runs)")
    ap.add_argument("--skip-anchored", action="store_true", help="leave out the anchor-guided alignment leg")
    ap.add_argument("--skip-configs", action="store_true",
                    help="leave out the 4,096-pair plain batch and the long-problem stress legs")
    ap.add_argument("--only-path", action="store_true",
                    help="run only the warping-path leg and print its JSON (for profiling runs)")
    ap.add_argument("--only-single-read", action="store_true",
                    help="run only the single-read latency leg and print its JSON")
    ap.add_argument("--only-banded", action="store_true",
                    help="run only the banded-DTW leg and print its JSON (for profiling runs)")
    ap.add_argument("--only-configs", action="store_true",
                    help="run only the 4,096-pair plain batch and long-stress legs (library defaults) and print them")
    ap.add_argument("--only-anchored", action="store_true",
                    help="run only the anchor-guided alignment leg and print its JSON (for profiling runs)")
    ap.add_argument("--only-early-termination", action="store_true",
                    help="run only the early-termination leg (library defaults, 512-row blocks) and print its JSON")
    ap.add_argument("--opts", type=str, default="", help="JSON dict of rawalign_opts fields for the tuned path")
    ap.add_argument("--no-autotune", action="store_true", help="time the library defaults instead of tuned settings")
    ap.add_argument("--serving-reads", type=int, default=20000, help="reads in the serving leg (0: skip it)")
    ap.add_argument("--serving-rate", type=float, default=2000.0)
    ap.add_argument("--serving-slots", type=int, default=3, help="serving ticks in flight")
    ap.add_argument("--serving-streams", type=int, default=3, choices=(1, 3),
                    help="library streams for the serving extension (3: the three route kernels concurrently)")
    ap.add_argument("--serving-pipe-waves", type=int, default=8, choices=(0, 2, 4, 8),
                    help="waves sharing each long region in the serving extension (0: one wave per pair)")
    ap.add_argument("--serving-single-max", type=int, default=2048, choices=(2048, 4096),
                    help="widest region swept as one stripe in the serving extension")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a copy kernel of this size (counter calibration)")
    ap.add_argument("--valu-rate", action="store_true",
                    help="only measure the VALU issue rate behind the roofline peak and print it")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.valu_rate:
        print(json.dumps({"valu_rate": valu_rate()}), flush=True)
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
    if args.only_single_read:
        print(json.dumps({"single_read": single_read_leg(lib)}), flush=True)
        return
    if args.only_early_termination:
        print(json.dumps({"early_termination": bnb_leg(lib, workloads.uneven_batch(), lib.make_opts(),
                                                       steps=args.steps)}), flush=True)
        return
    if args.only_path:
        print(json.dumps({"path": path_leg(lib, workloads.uneven_batch(), None, steps=args.steps)}), flush=True)
        return
    if args.only_configs:
        legs = {"plain_batch_4096": batch_config_leg(lib, workloads.plain_batch(), "plain_batch_4096_pairs",
                                                     valu_peak, {}, steps=10, warmup=2),
                "long_stress_1024": batch_config_leg(lib, workloads.long_stress(), "long_stress_1024_x_10000_x_20000",
                                                     valu_peak, {}, steps=args.steps, warmup=1, antidiag=True,
                                                     pipeline=True)}
        print(json.dumps({"configs": legs}), flush=True)
        return
    if args.only_banded:
        print(json.dumps({"banded": banded_leg(lib, valu_peak, steps=args.steps, warmup=args.warmup)}), flush=True)
        return

    b = workloads.uneven_batch()
    cells = b.cells
    db = lib.DeviceBatch(b)
    stream = torch.cuda.current_stream()

    extra = json.loads(args.opts) if args.opts else {}
    tune_ms = None
    if not args.no_autotune and not extra:
        # The library times its candidate launch settings on this batch and
        # keeps the fastest; the timed path uses it.
        t0 = time.perf_counter()
        note("autotune on the uneven batch")
        best = lib.rawalign_autotune(*db.args())
        tune_ms = (time.perf_counter() - t0) * 1e3
        extra = {k: v for k, v in best.as_dict().items() if k != "flags"}
    tuned = lib.make_opts(flags=lib.FLAG_TIMING, **extra)
    # The anti-diagonal kernel runs plain batches only: the legs that call
    # other entry points (alignment start, paths, early termination, banded)
    # take the striped kernel at its default grid when the tuner chose it,
    # as the library does for calls that inherit the tuned setting.
    extra_other = dict(extra)
    if int(extra_other.get("long_kernel", 0)) == lib.LONG_ANTIDIAG:
        extra_other.update(long_kernel=lib.LONG_STRIPED, long_waves_per_cu=0)
    single_max = int(extra.get("single_max") or 4096)
    rc = route_cells(b, single_max)
    long_name = {1: "k_antidiag", 2: "k_pipe"}.get(int(extra.get("long_kernel", 0)), "k_multi")
    plain_opts = lib.make_opts(mode=lib.MODE_PLAIN, flags=lib.FLAG_TIMING)

    def timed(opts, steps, warmup):
        return timed_steps(lib, db, opts, steps, warmup)

    note("timed steps")
    step_s, kt = timed(tuned, args.steps, args.warmup)
    gcups = cells / step_s / 1e9
    tuned_score, tuned_end = (x.copy() for x in db.results())
    checks = {}
    plain_gcups = plain_s = None
    pkt = {}
    variants = {}
    if not args.skip_plain:
        note("plain mode")
        plain_s, pkt = timed(plain_opts, max(2, args.steps // 2), 1)
        plain_gcups = cells / plain_s / 1e9
        ps, pe = db.results()
        # The timed (tuned, persistent) step must return the plain step's bits.
        checks["tuned_equals_plain_all_pairs"] = bool(
            np.array_equal(tuned_score.view(np.uint32), ps.view(np.uint32)) and np.array_equal(tuned_end, pe))
        # Same batch with the anti-diagonal kernel for the regions above one
        # stripe (the lane-striped kernels keep the shorter ones).
        ad_opts = lib.make_opts(flags=lib.FLAG_TIMING, long_kernel=lib.LONG_ANTIDIAG)
        note("anti-diagonal variant")
        ad_s, akt = timed(ad_opts, 2, 1)
        variants["long_antidiag"] = {"value": cells / ad_s / 1e9, "unit": "GCUPS", "ms_per_step": ad_s * 1e3,
                                     "kernels_ms": akt,
                                     "long_route_gcups": route_cells(b)["long"] / akt["long_ms"] / 1e6,
                                     "kernel": "k_antidiag"}
        # Same batch with the regions above one stripe shared by 4 waves each
        # (pipelined stripes), at the tuned cut-off.
        pp_opts = lib.make_opts(flags=lib.FLAG_TIMING, long_kernel=lib.LONG_PIPELINE, pipe_waves=4,
                                single_max=single_max)
        note("pipeline variant")
        pp_s, pkt4 = timed(pp_opts, 3, 1)
        variants["long_pipeline_4_waves"] = {"value": cells / pp_s / 1e9, "unit": "GCUPS",
                                             "ms_per_step": pp_s * 1e3, "kernels_ms": pkt4,
                                             "long_route_gcups": rc["long"] / pkt4["long_ms"] / 1e6,
                                             "kernel": "k_pipe", "single_max": single_max}

    if not args.skip_plain:
        note("early termination")
        variants["early_termination"] = bnb_leg(lib, b, lib.make_opts(**extra_other))
        note("alignment start")
        variants["alignment_start"] = span_leg(lib, db, lib.make_opts(**extra_other))
        note("warping paths")
        variants["path"] = path_leg(lib, b, lib.make_opts(**extra_other))
        checks["path_exact_workspace_paths_equal"] = variants["path"]["exact_workspace_paths_equal"]
        note("banded regions")
        variants["banded_regions"] = banded_regions_leg(lib, db, step_s * 1e3)
    if not args.skip_anchored:
        note("anchored alignment")
        variants["anchored"] = anchored_leg(lib, valu_peak)
    if not args.skip_plain:
        note("single read")
        variants["single_read"] = single_read_leg(lib)
    if not args.skip_anchored:
        note("banded chained segments")
        variants["banded"] = banded_leg(lib, valu_peak, lib.make_opts(**extra_other))
    configs = {}
    if not args.skip_configs:
        # the other batch workloads: the 4,096-pair plain batch and the
        # 1,024 x 10,000 x 20,000 long-problem stress
        del db
        torch.cuda.empty_cache()
        note("4,096-pair plain batch")
        configs["plain_batch_4096"] = batch_config_leg(lib, workloads.plain_batch(), "plain_batch_4096_pairs",
                                                      valu_peak, extra, steps=10, warmup=2)
        note("long stress")
        configs["long_stress_1024"] = batch_config_leg(lib, workloads.long_stress(),
                                                      "long_stress_1024_x_10000_x_20000", valu_peak, extra,
                                                      steps=3, warmup=1, antidiag=True, pipeline=True)
        for name, leg in configs.items():
            checks[f"{name}_forms_bit_identical"] = leg["all_forms_bit_identical"]

    # dominant kernel of the timed step: the route with the largest average duration
    names = {"lo_ms": "lo", "hi_ms": "hi", "long_ms": "long"}
    dom = max(names, key=lambda k: kt[k])
    dom_cells = rc[names[dom]]
    achieved = VALU_OPS_PER_CELL * dom_cells / (kt[dom] / 1e3)
    traffic = measured_traffic()
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": valu_peak / 1e12, "unit": "TOP/s",
                "frac": achieved / valu_peak, "traffic": traffic,
                "algorithmic_bytes": route_bytes(b, single_max)[names[dom]],
                "kernel": dict(KERNEL_NAMES, long_ms=long_name)[dom],
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
        "configs": configs,
        "checks": checks,
        "roofline": roofline,
        "serving": None,
        "cpu_baseline": None,
    }
    if "db" in locals():
        del db
    torch.cuda.empty_cache()
    if args.serving_reads > 0:
        note("serving")
        out["serving"] = serving_leg(args.serving_reads, args.serving_rate, args.serving_streams, args.serving_slots,
                                     pipe_waves=args.serving_pipe_waves, single_max=args.serving_single_max)
        checks["serving_capped_results_equal"] = out["serving"]["capped"]["results_equal_uncapped"]
    if not args.no_cpu:
        note("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(b, args.cpu_seconds, tuned_score, tuned_end)
        checks["oracle_sample_within_tolerance"] = out["cpu_baseline"]["parity"]["within_tolerance"]
    print(json.dumps(out), flush=True)
    failed = [k for k, v in checks.items() if not v]
    if failed:
        print(f"bench checks failed: {failed}", file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
