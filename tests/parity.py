"""Shared parity checks: GPU results against the CPU oracle.

The bar (tolerance of the score metric, 1e-4 relative): for every pair
  * |C_gpu - C_f64| <= 1e-4 * |C_f64| + 1e-6   (C_f64 from the double oracle);
  * C_gpu is bit-identical to the float oracle: every cell is one rounded
    subtraction, an exact |.|, an exact min and one rounded addition, so the
    float result does not depend on evaluation order;
  * end_gpu == end_f64 (smallest region index on ties).  Where float cannot
    resolve a near-tie of the double table the float end may differ; such a
    pair is accepted only if end_gpu equals the float oracle's end AND the
    double table's value at end_gpu is within the score tolerance of C_f64.
    Such pairs are counted and reported as float near-ties.
Sentinels (empty query / region, invalid slice) are compared exactly.
"""
from __future__ import annotations

import os

import numpy as np

from oracle import oracle

REL_TOL = 1e-4
ABS_TOL = 1e-6


def threads() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def oracle_batch(b, pairs=None):
    """Double and float oracle results for the pairs of a workloads.Batch."""
    if pairs is not None:
        b = b.subset(pairs)
    s64, e64, _ = oracle.dtw_batch_f64(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, threads())
    s32, e32, _ = oracle.dtw_batch_f32(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, threads())
    return s64, e64, s32, e32


def check(b, gpu_score, gpu_end, pairs=None, ref=None):
    """Assert parity for `pairs` (default: all) of batch b; returns stats."""
    gpu_score = np.asarray(gpu_score)
    gpu_end = np.asarray(gpu_end)
    if pairs is None:
        pairs = np.arange(b.n_pairs)
    pairs = np.asarray(pairs, dtype=np.int64)
    s64, e64, s32, e32 = ref if ref is not None else oracle_batch(b, pairs)
    gs = gpu_score[pairs]
    ge = gpu_end[pairs]
    # float oracle: bit-identical
    same = (gs.view(np.uint32) == s32.astype(np.float32).view(np.uint32)) | (np.isnan(gs) & np.isnan(s32))
    bad = np.nonzero(~same)[0]
    assert len(bad) == 0, (f"{len(bad)} pairs differ from the float oracle, e.g. pair {pairs[bad[0]]}: "
                           f"gpu {gs[bad[0]]!r} oracle {s32[bad[0]]!r}")
    assert np.array_equal(ge, e32), f"ends differ from the float oracle at pairs {pairs[np.nonzero(ge != e32)[0][:5]]}"
    # double oracle: relative tolerance
    fin = np.isfinite(s64)
    assert np.array_equal(np.isfinite(gs), fin)
    err = np.abs(gs[fin].astype(np.float64) - s64[fin])
    lim = REL_TOL * np.abs(s64[fin]) + ABS_TOL
    assert (err <= lim).all(), f"score error above tolerance: max rel {np.max(err / np.maximum(np.abs(s64[fin]), 1e-30)):.3g}"
    rel = err / np.maximum(np.abs(s64[fin]), 1e-30)
    # ends against the double oracle, with the near-tie protocol
    near_ties = 0
    for k in np.nonzero(ge != e64)[0]:
        p = int(pairs[k])
        q = b.q[b.q_off[p]:b.q_off[p] + b.q_len[p]]
        r = b.r[b.r_off[p]:b.r_off[p] + b.r_len[p]]
        c64, _, row = oracle.dtw_f64(q, r, want_row=True)
        j = int(ge[k])
        assert 0 <= j < len(r), f"pair {p}: end {j} outside the region"
        assert row[j] <= c64 * (1 + REL_TOL) + ABS_TOL, f"pair {p}: end {j} is not a near-optimal end"
        near_ties += 1
    return {"pairs": int(len(pairs)), "max_rel_err": float(rel.max()) if len(rel) else 0.0,
            "near_ties": near_ties}


def stratified_sample(b, k, seed=0):
    """k pairs spread over the cell-count distribution (includes the largest)."""
    cells = b.q_len.astype(np.int64) * b.r_len.astype(np.int64)
    order = np.argsort(cells)
    if k >= len(order):
        return order
    idx = np.unique(np.linspace(0, len(order) - 1, k).round().astype(np.int64))
    return np.sort(order[idx])
