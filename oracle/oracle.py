"""CPU oracle for RawAlign's alignment step (arXiv 2310.05037).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the HIP library.

* ``dtw_f64`` / ``dtw_f32`` / ``dtw_batch_*``: subsequence DTW of Sec. 2.2
  (cell cost = numerical difference, three neighbours, no indel penalty,
  query aligned whole, free start and end in the region), computed by the
  plain C recurrence in ``dtw_oracle.c``.
* ``decide``: the mapping decision of Sec. 2.3: Score = B_Match * N_Read -
  C_DTW per candidate, the highest score of a read is mapped iff it is at
  least Score_Threshold (defaults 0.4 and 20 from Sec. 3.1.5).
* ``dtw_span_*``: subsequence DTW with the start of the alignment (the
  path's first region column; Sec. 2.4 lets the path be added to the
  output): the read aligned backwards against the region prefix ending at
  the end column, anchored there, free to finish anywhere; ties give the
  largest start (the shortest optimal alignment).
* ``dtw_band_*``: banded subsequence DTW of Sec. 2.4.3: cells farther than
  w levels from the diagonal column floor(i*m/n) are +inf.
* ``dtw_global_*`` / ``chain_costs`` / ``decide_chains``: anchor-guided
  alignment of Sec. 2.4.2: every gap between two consecutive anchors of a
  chain is aligned by global DTW entered and left through the anchor corners;
  a chain's cost is the sum of its gaps' costs, taken in gap order; its Score
  is B_Match times the events the chain aligns minus that cost.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dtw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

B_MATCH = 0.4  # Sec. 3.1.5 parameter settings
SCORE_THRESHOLD = 20.0  # Sec. 3.1.5 parameter settings


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc: -O2, IEEE semantics, no contraction."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64 = ctypes.c_int64
        L.oracle_dtw_f64.restype = ctypes.c_double
        L.oracle_dtw_f64.argtypes = [f32p, i64, f32p, i64, f64p, f64p, i32p]
        L.oracle_dtw_f32.restype = ctypes.c_float
        L.oracle_dtw_f32.argtypes = [f32p, i64, f32p, i64, f32p, f32p, i32p]
        L.oracle_dtw_matrix_f64.restype = None
        L.oracle_dtw_matrix_f64.argtypes = [f32p, i64, f32p, i64, f64p]
        for name, outp in (("oracle_dtw_batch_f64", f64p), ("oracle_dtw_batch_f32", f32p)):
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [f32p, i64p, i32p, f32p, i64p, i32p, i64, outp, i32p, ctypes.c_int]
        L.oracle_dtw_band_f64.restype = ctypes.c_double
        L.oracle_dtw_band_f64.argtypes = [f32p, i64, f32p, i64, i64, i32p]
        L.oracle_dtw_band_f32.restype = ctypes.c_float
        L.oracle_dtw_band_f32.argtypes = [f32p, i64, f32p, i64, i64, i32p]
        for name, outp in (("oracle_dtw_band_batch_f64", f64p), ("oracle_dtw_band_batch_f32", f32p)):
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [f32p, i64p, i32p, f32p, i64p, i32p, i32p, i64, outp, i32p, ctypes.c_int]
        L.oracle_dtw_span_f64.restype = ctypes.c_double
        L.oracle_dtw_span_f64.argtypes = [f32p, i64, f32p, i64, i32p, i32p]
        L.oracle_dtw_span_f32.restype = ctypes.c_float
        L.oracle_dtw_span_f32.argtypes = [f32p, i64, f32p, i64, i32p, i32p]
        for name, outp in (("oracle_dtw_span_batch_f64", f64p), ("oracle_dtw_span_batch_f32", f32p)):
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [f32p, i64p, i32p, f32p, i64p, i32p, i64, outp, i32p, i32p, ctypes.c_int]
        L.oracle_dtw_path_f64.restype = ctypes.c_double
        L.oracle_dtw_path_f64.argtypes = [f32p, i64, f32p, ctypes.c_int32, ctypes.c_int32, i32p, i32p]
        L.oracle_dtw_path_f32.restype = ctypes.c_float
        L.oracle_dtw_path_f32.argtypes = [f32p, i64, f32p, ctypes.c_int32, ctypes.c_int32, i32p, i32p]
        L.oracle_dtw_global_f64.restype = ctypes.c_double
        L.oracle_dtw_global_f64.argtypes = [f32p, i64, f32p, i64]
        L.oracle_dtw_global_f32.restype = ctypes.c_float
        L.oracle_dtw_global_f32.argtypes = [f32p, i64, f32p, i64]
        for name, outp in (("oracle_dtw_global_batch_f64", f64p), ("oracle_dtw_global_batch_f32", f32p)):
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [f32p, i64p, i32p, f32p, i64p, i32p, i64, outp, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _f32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32))


def dtw_f64(q, r, init_row=None, want_row: bool = False):
    """One pair in double precision -> (cost, end[, last_row])."""
    q = _f32(q)
    r = _f32(r)
    end = ctypes.c_int32(0)
    row = np.empty(len(r), dtype=np.float64) if want_row else None
    ir = None
    if init_row is not None:
        ir = np.ascontiguousarray(np.asarray(init_row, dtype=np.float64))
        assert len(ir) == len(r)
    c = lib().oracle_dtw_f64(_ptr(q, ctypes.c_float), len(q), _ptr(r, ctypes.c_float), len(r),
                             None if ir is None else _ptr(ir, ctypes.c_double),
                             None if row is None else _ptr(row, ctypes.c_double),
                             ctypes.byref(end))
    return (c, end.value, row) if want_row else (c, end.value)


def dtw_f32(q, r, init_row=None, want_row: bool = False):
    """One pair with every value in float -> (cost, end[, last_row])."""
    q = _f32(q)
    r = _f32(r)
    end = ctypes.c_int32(0)
    row = np.empty(len(r), dtype=np.float32) if want_row else None
    ir = None
    if init_row is not None:
        ir = _f32(init_row)
        assert len(ir) == len(r)
    c = lib().oracle_dtw_f32(_ptr(q, ctypes.c_float), len(q), _ptr(r, ctypes.c_float), len(r),
                             None if ir is None else _ptr(ir, ctypes.c_float),
                             None if row is None else _ptr(row, ctypes.c_float),
                             ctypes.byref(end))
    c = np.float32(c)
    return (c, end.value, row) if want_row else (c, end.value)


def dtw_matrix_f64(q, r) -> np.ndarray:
    """Full n x m table D(i, j) for small inputs."""
    q = _f32(q)
    r = _f32(r)
    D = np.empty((len(q), len(r)), dtype=np.float64)
    if len(q) and len(r):
        lib().oracle_dtw_matrix_f64(_ptr(q, ctypes.c_float), len(q), _ptr(r, ctypes.c_float),
                                    len(r), _ptr(D, ctypes.c_double))
    return D


def _batch(fn, dtype, q, q_off, q_len, r, r_off, r_len, threads):
    q = _f32(q)
    r = _f32(r)
    q_off = np.ascontiguousarray(q_off, dtype=np.int64)
    r_off = np.ascontiguousarray(r_off, dtype=np.int64)
    q_len = np.ascontiguousarray(q_len, dtype=np.int32)
    r_len = np.ascontiguousarray(r_len, dtype=np.int32)
    n = len(q_off)
    assert len(q_len) == n and len(r_off) == n and len(r_len) == n
    assert n == 0 or (int((q_off + q_len).max()) <= len(q) and int(q_off.min()) >= 0)
    assert n == 0 or (int((r_off + r_len).max()) <= len(r) and int(r_off.min()) >= 0)
    score = np.empty(n, dtype=dtype)
    end = np.empty(n, dtype=np.int32)
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    used = 0
    if n:
        ct = ctypes.c_double if dtype == np.float64 else ctypes.c_float
        used = fn(_ptr(q, ctypes.c_float), _ptr(q_off, ctypes.c_int64), _ptr(q_len, ctypes.c_int32),
                  _ptr(r, ctypes.c_float), _ptr(r_off, ctypes.c_int64), _ptr(r_len, ctypes.c_int32),
                  n, _ptr(score, ct), _ptr(end, ctypes.c_int32), int(threads))
    return score, end, used


def dtw_batch_f64(q, q_off, q_len, r, r_off, r_len, threads=None):
    """Batch in double precision -> (scores f64, ends i32, threads used)."""
    return _batch(lib().oracle_dtw_batch_f64, np.float64, q, q_off, q_len, r, r_off, r_len, threads)


def dtw_batch_f32(q, q_off, q_len, r, r_off, r_len, threads=None):
    """Batch with float arithmetic -> (scores f32, ends i32, threads used)."""
    return _batch(lib().oracle_dtw_batch_f32, np.float32, q, q_off, q_len, r, r_off, r_len, threads)


def decide(cost, cand_off, cand_cnt, n_events, b_match=B_MATCH, threshold=SCORE_THRESHOLD):
    """Mapping decision of Sec. 2.3, one read at a time.

    cost[p] is C_DTW of pair p (taken in the precision it was computed in and
    widened to double); read k owns pairs cand_off[k] .. cand_off[k]+cand_cnt[k]-1
    and has n_events[k] aligned read events.  Score = b_match*N_Read - C_DTW
    in double precision.  The best candidate is the highest score, the
    smallest pair index on ties; the read is mapped iff that score >= threshold.
    A NaN cost marks a pair that was not aligned (an invalid or unsupported
    pair): it is not a candidate.
    Returns (best pair index or -1, best score or -inf, mapped flag).
    """
    n_reads = len(cand_off)
    best = np.full(n_reads, -1, dtype=np.int32)
    best_score = np.full(n_reads, -np.inf, dtype=np.float64)
    mapped = np.zeros(n_reads, dtype=np.uint8)
    for k in range(n_reads):
        N = float(n_events[k])
        for p in range(int(cand_off[k]), int(cand_off[k]) + int(cand_cnt[k])):
            if np.isnan(cost[p]):
                continue
            s = b_match * N - float(cost[p])
            if best[k] < 0 or s > best_score[k]:
                best[k] = p
                best_score[k] = s
        if best[k] >= 0 and best_score[k] >= threshold:
            mapped[k] = 1
    return best, best_score, mapped


# ---- anchor-guided alignment (Sec. 2.4.2) ---------------------------------------

def dtw_global_f64(q, r) -> float:
    """Global DTW of one gap, entered and left through the anchor corners
    (D(-1,-1) = 0, the rest of row -1 and column -1 +inf, result D(n-1, m-1));
    0 when both sides are empty, +inf when only one is."""
    q = _f32(q)
    r = _f32(r)
    return float(lib().oracle_dtw_global_f64(_ptr(q, ctypes.c_float), len(q), _ptr(r, ctypes.c_float), len(r)))


def dtw_global_f32(q, r) -> np.float32:
    """The same recurrence with every value in float."""
    q = _f32(q)
    r = _f32(r)
    return np.float32(lib().oracle_dtw_global_f32(_ptr(q, ctypes.c_float), len(q), _ptr(r, ctypes.c_float),
                                                  len(r)))


def _global_batch(fn, dtype, q, q_off, q_len, r, r_off, r_len, threads):
    q = _f32(q)
    r = _f32(r)
    q_off = np.ascontiguousarray(q_off, dtype=np.int64)
    r_off = np.ascontiguousarray(r_off, dtype=np.int64)
    q_len = np.ascontiguousarray(q_len, dtype=np.int32)
    r_len = np.ascontiguousarray(r_len, dtype=np.int32)
    n = len(q_off)
    assert len(q_len) == n and len(r_off) == n and len(r_len) == n
    assert n == 0 or (int((q_off + q_len).max()) <= len(q) and int(q_off.min()) >= 0)
    assert n == 0 or (int((r_off + r_len).max()) <= len(r) and int(r_off.min()) >= 0)
    out = np.empty(n, dtype=dtype)
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    used = 0
    if n:
        ct = ctypes.c_double if dtype == np.float64 else ctypes.c_float
        used = fn(_ptr(q, ctypes.c_float), _ptr(q_off, ctypes.c_int64), _ptr(q_len, ctypes.c_int32),
                  _ptr(r, ctypes.c_float), _ptr(r_off, ctypes.c_int64), _ptr(r_len, ctypes.c_int32),
                  n, _ptr(out, ct), int(threads))
    return out, used


def dtw_global_batch_f64(q, q_off, q_len, r, r_off, r_len, threads=None):
    """Global DTW of every pair in double precision -> (costs f64, threads used)."""
    return _global_batch(lib().oracle_dtw_global_batch_f64, np.float64, q, q_off, q_len, r, r_off, r_len, threads)


def dtw_global_batch_f32(q, q_off, q_len, r, r_off, r_len, threads=None):
    """Global DTW of every pair with float arithmetic -> (costs f32, threads used)."""
    return _global_batch(lib().oracle_dtw_global_batch_f32, np.float32, q, q_off, q_len, r, r_off, r_len, threads)


def chain_costs(gap_cost, chain_gap_off, chain_gap_cnt):
    """Cost of every chain: the sum of its gaps' costs, added one gap after
    another in gap order in the precision of `gap_cost` (float32 sums stay
    float32).  A chain without gaps (a single anchor) costs 0; a chain whose
    gap range leaves the gap array gets NaN."""
    gap_cost = np.asarray(gap_cost)
    dt = gap_cost.dtype.type
    out = np.empty(len(chain_gap_off), dtype=gap_cost.dtype)
    for c in range(len(chain_gap_off)):
        g0, cnt = int(chain_gap_off[c]), int(chain_gap_cnt[c])
        if cnt < 0 or g0 < 0 or g0 + cnt > len(gap_cost):
            out[c] = np.nan
            continue
        acc = dt(0)
        for g in range(g0, g0 + cnt):
            acc = dt(acc + gap_cost[g])
        out[c] = acc
    return out


def decide_chains(chain_cost, chain_events, cand_off, cand_cnt, b_match=B_MATCH, threshold=SCORE_THRESHOLD):
    """Mapping decision of Sec. 2.3 over anchored candidates: candidate c of a
    read scores b_match * chain_events[c] - chain_cost[c] (double precision),
    where chain_events[c] counts the read events its chain aligns; the
    highest score wins, the smallest candidate index on ties, and the read is
    mapped iff that score >= threshold.  A chain whose cost is NaN (a gap
    range outside the gap array, or an invalid gap) is not a candidate."""
    n_reads = len(cand_off)
    best = np.full(n_reads, -1, dtype=np.int32)
    best_score = np.full(n_reads, -np.inf, dtype=np.float64)
    mapped = np.zeros(n_reads, dtype=np.uint8)
    for k in range(n_reads):
        for c in range(int(cand_off[k]), int(cand_off[k]) + int(cand_cnt[k])):
            if np.isnan(chain_cost[c]):
                continue
            s = b_match * float(chain_events[c]) - float(chain_cost[c])
            if best[k] < 0 or s > best_score[k]:
                best[k] = c
                best_score[k] = s
        if best[k] >= 0 and best_score[k] >= threshold:
            mapped[k] = 1
    return best, best_score, mapped


# ---- start of the alignment ------------------------------------------------------

def dtw_span_f64(q, r):
    """(C_DTW, end, start) in double precision; start -1 with end -1."""
    q = _f32(q)
    r = _f32(r)
    e, st = ctypes.c_int32(0), ctypes.c_int32(0)
    c = lib().oracle_dtw_span_f64(_ptr(q, ctypes.c_float), len(q), _ptr(r, ctypes.c_float), len(r),
                                  ctypes.byref(e), ctypes.byref(st))
    return c, e.value, st.value


def dtw_span_f32(q, r):
    """The same with every value in float."""
    q = _f32(q)
    r = _f32(r)
    e, st = ctypes.c_int32(0), ctypes.c_int32(0)
    c = lib().oracle_dtw_span_f32(_ptr(q, ctypes.c_float), len(q), _ptr(r, ctypes.c_float), len(r),
                                  ctypes.byref(e), ctypes.byref(st))
    return np.float32(c), e.value, st.value


def _path(fn, span, cast, q, r):
    q = _f32(q)
    r = _f32(r)
    c, e, st = span(q, r)
    n = len(q)
    lo = np.full(n, -1, dtype=np.int32)
    hi = np.full(n, -1, dtype=np.int32)
    if e < 0:
        return c, e, st, cast(np.nan if e < -1 else c), lo, hi
    g = fn(_ptr(q, ctypes.c_float), n, _ptr(r, ctypes.c_float), st, e, _ptr(lo, ctypes.c_int32),
           _ptr(hi, ctypes.c_int32))
    return c, e, st, cast(g), lo, hi


def dtw_path_f64(q, r):
    """Subsequence DTW with its warping path, double precision (Sec. 2.4):
    (C_DTW, end, start, path cost, lo, hi) where read event i is aligned with
    region levels lo[i] .. hi[i] on an optimal path from (0, start) to
    (n-1, end); the path cost is the global cost of [start, end].  Empty
    query or region: lo = hi = -1."""
    return _path(lib().oracle_dtw_path_f64, dtw_span_f64, float, q, r)


def dtw_path_f32(q, r):
    """The same with every value in float (start from the float reverse
    pass, path from the float table)."""
    return _path(lib().oracle_dtw_path_f32, dtw_span_f32, np.float32, q, r)


def _span_batch(fn, dtype, q, q_off, q_len, r, r_off, r_len, threads):
    q = _f32(q)
    r = _f32(r)
    q_off = np.ascontiguousarray(q_off, dtype=np.int64)
    r_off = np.ascontiguousarray(r_off, dtype=np.int64)
    q_len = np.ascontiguousarray(q_len, dtype=np.int32)
    r_len = np.ascontiguousarray(r_len, dtype=np.int32)
    n = len(q_off)
    assert len(q_len) == n and len(r_off) == n and len(r_len) == n
    assert n == 0 or (int((q_off + q_len).max()) <= len(q) and int(q_off.min()) >= 0)
    assert n == 0 or (int((r_off + r_len).max()) <= len(r) and int(r_off.min()) >= 0)
    score = np.empty(n, dtype=dtype)
    end = np.empty(n, dtype=np.int32)
    start = np.empty(n, dtype=np.int32)
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    if n:
        ct = ctypes.c_double if dtype == np.float64 else ctypes.c_float
        fn(_ptr(q, ctypes.c_float), _ptr(q_off, ctypes.c_int64), _ptr(q_len, ctypes.c_int32),
           _ptr(r, ctypes.c_float), _ptr(r_off, ctypes.c_int64), _ptr(r_len, ctypes.c_int32),
           n, _ptr(score, ct), _ptr(end, ctypes.c_int32), _ptr(start, ctypes.c_int32), int(threads))
    return score, end, start


def dtw_span_batch_f64(q, q_off, q_len, r, r_off, r_len, threads=None):
    """(scores f64, ends, starts) of every pair."""
    return _span_batch(lib().oracle_dtw_span_batch_f64, np.float64, q, q_off, q_len, r, r_off, r_len, threads)


def dtw_span_batch_f32(q, q_off, q_len, r, r_off, r_len, threads=None):
    """(scores f32, ends, starts) of every pair with float arithmetic."""
    return _span_batch(lib().oracle_dtw_span_batch_f32, np.float32, q, q_off, q_len, r, r_off, r_len, threads)


# ---- banded alignment (Sec. 2.4.3) -------------------------------------------------

def dtw_band_f64(q, r, w):
    """(C_DTW, end) of banded subsequence DTW with half-width w, double."""
    q = _f32(q)
    r = _f32(r)
    e = ctypes.c_int32(0)
    c = lib().oracle_dtw_band_f64(_ptr(q, ctypes.c_float), len(q), _ptr(r, ctypes.c_float), len(r), int(w),
                                  ctypes.byref(e))
    return c, e.value


def dtw_band_f32(q, r, w):
    """The same with every value in float."""
    q = _f32(q)
    r = _f32(r)
    e = ctypes.c_int32(0)
    c = lib().oracle_dtw_band_f32(_ptr(q, ctypes.c_float), len(q), _ptr(r, ctypes.c_float), len(r), int(w),
                                  ctypes.byref(e))
    return np.float32(c), e.value


def _band_batch(fn, dtype, q, q_off, q_len, r, r_off, r_len, band, threads):
    q = _f32(q)
    r = _f32(r)
    q_off = np.ascontiguousarray(q_off, dtype=np.int64)
    r_off = np.ascontiguousarray(r_off, dtype=np.int64)
    q_len = np.ascontiguousarray(q_len, dtype=np.int32)
    r_len = np.ascontiguousarray(r_len, dtype=np.int32)
    band = np.ascontiguousarray(band, dtype=np.int32)
    n = len(q_off)
    assert len(q_len) == n and len(r_off) == n and len(r_len) == n and len(band) == n
    score = np.empty(n, dtype=dtype)
    end = np.empty(n, dtype=np.int32)
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    if n:
        ct = ctypes.c_double if dtype == np.float64 else ctypes.c_float
        fn(_ptr(q, ctypes.c_float), _ptr(q_off, ctypes.c_int64), _ptr(q_len, ctypes.c_int32),
           _ptr(r, ctypes.c_float), _ptr(r_off, ctypes.c_int64), _ptr(r_len, ctypes.c_int32),
           _ptr(band, ctypes.c_int32), n, _ptr(score, ct), _ptr(end, ctypes.c_int32), int(threads))
    return score, end


def dtw_band_batch_f64(q, q_off, q_len, r, r_off, r_len, band, threads=None):
    return _band_batch(lib().oracle_dtw_band_batch_f64, np.float64, q, q_off, q_len, r, r_off, r_len, band, threads)


def dtw_band_batch_f32(q, q_off, q_len, r, r_off, r_len, band, threads=None):
    return _band_batch(lib().oracle_dtw_band_batch_f32, np.float32, q, q_off, q_len, r, r_off, r_len, band, threads)
