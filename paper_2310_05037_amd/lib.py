"""ctypes binding of librawalign.so (C ABI in include/rawalign.h).

Argument marshalling only: every entry point takes torch CUDA tensors, checks
their device, dtype and contiguity on the host, and passes raw device
pointers plus the current HIP stream to the library function of the same
name.  All computation happens in the library's HIP kernels; there is no
fallback.  If the library is missing, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librawalign.so")

RAWALIGN_OK = 0
RAWALIGN_EINVAL = -1
RAWALIGN_EHIP = -2
RAWALIGN_ENOMEM = -3
RAWALIGN_ENODEV = -4
RAWALIGN_MAX_REGION = 65536
RAWALIGN_MAX_QUERY_LONG = 16384
RAWALIGN_NOALLOC_MAX_PAIRS = 131072
RAWALIGN_NOALLOC_EDGE_SLOTS = 512
MODE_PLAIN = 0
MODE_PERSISTENT = 1
LONG_STRIPED = 0
LONG_ANTIDIAG = 1
LONG_PIPELINE = 2
FLAG_TIMING = 1
FLAG_SPAN_GIVEN = 2   # rawalign_dtw_path: the span outputs are inputs (see path_workspace_exact)

# Every symbol include/rawalign.h declares.
EXPORTS = (
    "rawalign_opts_default", "rawalign_dtw_batch", "rawalign_dtw_batch_ex", "rawalign_dtw_batch_noalloc",
    "rawalign_dtw_extend",
    "rawalign_decide", "rawalign_map_bnb", "rawalign_dtw_span", "rawalign_dtw_path", "rawalign_dtw_band",
    "rawalign_dtw_global_batch",
    "rawalign_chain_decide",
    "rawalign_autotune", "rawalign_load_tuning", "rawalign_last_timing", "rawalign_last_error", "rawalign_version",
)


class RawAlignError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"librawalign error {code}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("long_kernel", ctypes.c_int32), ("lo_waves_per_cu", ctypes.c_int32),
                ("hi_waves_per_cu", ctypes.c_int32), ("long_waves_per_cu", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("flags", ctypes.c_int32), ("single_max", ctypes.c_int32),
                ("pipe_waves", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Timing(ctypes.Structure):
    _fields_ = [("plan_ms", ctypes.c_float), ("lo_ms", ctypes.c_float), ("hi_ms", ctypes.c_float),
                ("long_ms", ctypes.c_float), ("total_ms", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {k: float(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load librawalign.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    # torch first: the library then binds to the HIP runtime torch already
    # loaded, so device memory and streams from torch are valid in it.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    pair_args = [vp, i64, vp, vp, vp, i64, vp, vp, i64, vp, vp, vp]
    L.rawalign_opts_default.argtypes = [ctypes.POINTER(Opts)]
    L.rawalign_dtw_batch.argtypes = pair_args
    L.rawalign_dtw_batch_ex.argtypes = pair_args + [ctypes.POINTER(Opts)]
    L.rawalign_dtw_batch_noalloc.argtypes = pair_args
    L.rawalign_dtw_extend.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp, vp, i64, vp, vp, i64, vp, vp, vp,
                                      ctypes.POINTER(Opts)]
    L.rawalign_decide.argtypes = [vp, i64, vp, vp, vp, i64, f64, f64, vp, vp, vp, vp]
    L.rawalign_map_bnb.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp, i64, vp, vp, vp, i64, f64, f64, i32, i32,
                                   vp, i64, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Opts)]
    L.rawalign_dtw_global_batch.argtypes = pair_args + [ctypes.POINTER(Opts)]
    L.rawalign_dtw_span.argtypes = pair_args[:11] + [vp, vp, ctypes.POINTER(Opts)]
    L.rawalign_dtw_path.argtypes = pair_args[:9] + [vp, vp, i64, vp, vp, vp, i64, vp, vp, vp, vp,
                                                    ctypes.POINTER(Opts)]
    L.rawalign_dtw_band.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp, vp, i64, vp, vp, vp]
    L.rawalign_chain_decide.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp, i64, f64, f64, vp, vp, vp, vp, vp]
    L.rawalign_autotune.argtypes = pair_args + [ctypes.c_char_p, ctypes.POINTER(Opts)]
    L.rawalign_load_tuning.argtypes = [ctypes.c_char_p, ctypes.POINTER(Opts)]
    L.rawalign_last_timing.argtypes = [ctypes.POINTER(Timing)]
    L.rawalign_last_error.restype = ctypes.c_char_p
    L.rawalign_last_error.argtypes = []
    L.rawalign_version.restype = ctypes.c_char_p
    L.rawalign_version.argtypes = []
    for name in EXPORTS:
        if name not in ("rawalign_last_error", "rawalign_version"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != RAWALIGN_OK:
        raise RawAlignError(rc, load().rawalign_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _pair_args(q, q_off, q_len, r, r_off, r_len, out_score, out_end):
    """out_end may be None only where the entry point allows it."""
    import torch
    n = q_off.numel()
    for t, nm in ((q_len, "q_len"), (r_off, "r_off"), (r_len, "r_len"), (out_score, "out_score"),
                  (out_end, "out_end")):
        if t is not None and t.numel() != n:
            raise ValueError(f"{nm} has {t.numel()} elements, expected {n}")
    return [_dev(q, torch.float32, "q"), q.numel(), _dev(q_off, torch.int64, "q_off"),
            _dev(q_len, torch.int32, "q_len"), _dev(r, torch.float32, "r"), r.numel(),
            _dev(r_off, torch.int64, "r_off"), _dev(r_len, torch.int32, "r_len"), n,
            _dev(out_score, torch.float32, "out_score"),
            None if out_end is None else _dev(out_end, torch.int32, "out_end")]


def opts_default() -> Opts:
    o = Opts()
    _check(load().rawalign_opts_default(ctypes.byref(o)))
    return o


def make_opts(**kw) -> Opts:
    o = opts_default()
    names = {f for f, _ in Opts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise ValueError(f"rawalign_opts has no field {k!r}")
        setattr(o, k, int(v))
    return o


def rawalign_dtw_batch(q, q_off, q_len, r, r_off, r_len, out_score, out_end, stream=None):
    _check(load().rawalign_dtw_batch(*_pair_args(q, q_off, q_len, r, r_off, r_len, out_score, out_end),
                                     _stream(stream)))


def rawalign_dtw_batch_ex(q, q_off, q_len, r, r_off, r_len, out_score, out_end, opts=None, stream=None):
    _check(load().rawalign_dtw_batch_ex(*_pair_args(q, q_off, q_len, r, r_off, r_len, out_score, out_end),
                                        _stream(stream), None if opts is None else ctypes.byref(opts)))


def rawalign_dtw_batch_noalloc(q, q_off, q_len, r, r_off, r_len, out_score, out_end, stream=None):
    _check(load().rawalign_dtw_batch_noalloc(*_pair_args(q, q_off, q_len, r, r_off, r_len, out_score, out_end),
                                             _stream(stream)))


def rawalign_dtw_extend(q, q_off, q_len, r, r_off, r_len, rows, row_off, first_chunk, out_score, out_end,
                        opts=None, stream=None):
    import torch
    a = _pair_args(q, q_off, q_len, r, r_off, r_len, out_score, out_end)
    n = a[8]
    if row_off.numel() != n or first_chunk.numel() != n:
        raise ValueError("row_off and first_chunk need one entry per job")
    _check(load().rawalign_dtw_extend(*a[:8], _dev(rows, torch.float32, "rows"), rows.numel(),
                                      _dev(row_off, torch.int64, "row_off"),
                                      _dev(first_chunk, torch.uint8, "first_chunk"), n, a[9], a[10],
                                      _stream(stream), None if opts is None else ctypes.byref(opts)))


def rawalign_map_bnb(q, q_off, q_len, r, r_off, r_len, cand_off, cand_cnt, n_events, rows, row_off,
                     out_score, out_end, out_best, out_best_score, out_mapped, max_query, block_rows=512,
                     b_match=0.4, threshold=20.0, opts=None, stream=None):
    import torch
    a = _pair_args(q, q_off, q_len, r, r_off, r_len, out_score, out_end)
    n = a[8]
    n_reads = cand_off.numel()
    if row_off.numel() != n:
        raise ValueError("row_off needs one entry per pair")
    for t, nm in ((cand_cnt, "cand_cnt"), (n_events, "n_events"), (out_best, "out_best"),
                  (out_best_score, "out_best_score"), (out_mapped, "out_mapped")):
        if t.numel() != n_reads:
            raise ValueError(f"{nm} has {t.numel()} elements, expected {n_reads}")
    _check(load().rawalign_map_bnb(*a[:9], _dev(cand_off, torch.int64, "cand_off"),
                                   _dev(cand_cnt, torch.int32, "cand_cnt"), _dev(n_events, torch.int32, "n_events"),
                                   n_reads, float(b_match), float(threshold), int(max_query), int(block_rows),
                                   _dev(rows, torch.float32, "rows"), rows.numel(),
                                   _dev(row_off, torch.int64, "row_off"), a[9], a[10],
                                   _dev(out_best, torch.int32, "out_best"),
                                   _dev(out_best_score, torch.float64, "out_best_score"),
                                   _dev(out_mapped, torch.uint8, "out_mapped"), _stream(stream),
                                   None if opts is None else ctypes.byref(opts)))


def rawalign_decide(score, cand_off, cand_cnt, n_events, out_best, out_score, out_mapped,
                    b_match=0.4, threshold=20.0, stream=None):
    import torch
    n_reads = cand_off.numel()
    for t, nm in ((cand_cnt, "cand_cnt"), (n_events, "n_events"), (out_best, "out_best"),
                  (out_score, "out_score"), (out_mapped, "out_mapped")):
        if t.numel() != n_reads:
            raise ValueError(f"{nm} has {t.numel()} elements, expected {n_reads}")
    _check(load().rawalign_decide(_dev(score, torch.float32, "score"), score.numel(),
                                  _dev(cand_off, torch.int64, "cand_off"), _dev(cand_cnt, torch.int32, "cand_cnt"),
                                  _dev(n_events, torch.int32, "n_events"), n_reads, float(b_match),
                                  float(threshold), _dev(out_best, torch.int32, "out_best"),
                                  _dev(out_score, torch.float64, "out_score"),
                                  _dev(out_mapped, torch.uint8, "out_mapped"), _stream(stream)))


def rawalign_dtw_span(q, q_off, q_len, r, r_off, r_len, out_score, out_end, out_start, opts=None, stream=None):
    import torch
    a = _pair_args(q, q_off, q_len, r, r_off, r_len, out_score, out_end)
    if out_start.numel() != a[8]:
        raise ValueError(f"out_start has {out_start.numel()} elements, expected {a[8]}")
    _check(load().rawalign_dtw_span(*a, _dev(out_start, torch.int32, "out_start"), _stream(stream),
                                    None if opts is None else ctypes.byref(opts)))


def path_workspace(q_len, r_len):
    """(dir_off, words) of a direction workspace that holds the path of every
    pair: n * (64 * ceil(m / 2048) + 1) 64-bit words per pair (numpy int64
    offsets; the interval of an alignment is at most m levels)."""
    n = np.maximum(np.asarray(q_len, dtype=np.int64), 0)
    m = np.maximum(np.asarray(r_len, dtype=np.int64), 1)
    words = n * (64 * ((m + 2047) // 2048) + 1)
    off = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.int64)
    return off, int(words.sum())


def path_workspace_exact(q_len, out_end, out_start):
    """(dir_off, words) of a direction workspace sized from the intervals of
    a rawalign_dtw_span call: n * (64 * ceil(L / 2048) + 1) 64-bit words for
    a pair aligned over L = end - start + 1 levels, none for a pair without
    an alignment.  Pass it to rawalign_dtw_path with FLAG_SPAN_GIVEN and the
    same span outputs."""
    n = np.maximum(np.asarray(q_len, dtype=np.int64), 0)
    e = np.asarray(out_end, dtype=np.int64)
    st = np.asarray(out_start, dtype=np.int64)
    ok = (e >= 0) & (st >= 0) & (st <= e)
    L = np.where(ok, e - st + 1, 0)
    words = np.where(ok, n * (64 * ((L + 2047) // 2048) + 1), 0)
    off = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.int64)
    return off, int(words.sum())


def rawalign_dtw_path(q, q_off, q_len, r, r_off, r_len, dir_off, dirs, path_off, path_lo, path_hi, out_score,
                      out_end, out_start, opts=None, stream=None):
    """dirs: int64 CUDA tensor (the 64-bit direction words), dir_off: int64
    per pair (see path_workspace)."""
    import torch
    a = _pair_args(q, q_off, q_len, r, r_off, r_len, out_score, out_end)
    n = a[8]
    for t, nm in ((dir_off, "dir_off"), (path_off, "path_off"), (out_start, "out_start")):
        if t.numel() != n:
            raise ValueError(f"{nm} has {t.numel()} elements, expected {n}")
    if path_lo.numel() != path_hi.numel():
        raise ValueError("path_lo and path_hi must have the same size")
    _check(load().rawalign_dtw_path(*a[:9], _dev(dir_off, torch.int64, "dir_off"), _dev(dirs, torch.int64, "dirs"),
                                    dirs.numel(), _dev(path_off, torch.int64, "path_off"),
                                    _dev(path_lo, torch.int32, "path_lo"), _dev(path_hi, torch.int32, "path_hi"),
                                    path_lo.numel(), a[9], a[10], _dev(out_start, torch.int32, "out_start"),
                                    _stream(stream), None if opts is None else ctypes.byref(opts)))


def rawalign_dtw_band(q, q_off, q_len, r, r_off, r_len, band, out_score, out_end, stream=None):
    import torch
    a = _pair_args(q, q_off, q_len, r, r_off, r_len, out_score, out_end)
    if band.numel() != a[8]:
        raise ValueError(f"band has {band.numel()} elements, expected {a[8]}")
    _check(load().rawalign_dtw_band(*a[:8], _dev(band, torch.int32, "band"), a[8], a[9], a[10], _stream(stream)))


def rawalign_dtw_global_batch(q, q_off, q_len, r, r_off, r_len, out_score, out_end=None, opts=None, stream=None):
    _check(load().rawalign_dtw_global_batch(*_pair_args(q, q_off, q_len, r, r_off, r_len, out_score, out_end),
                                            _stream(stream), None if opts is None else ctypes.byref(opts)))


def rawalign_chain_decide(gap_cost, chain_gap_off, chain_gap_cnt, chain_events, cand_off, cand_cnt,
                          out_chain_cost, out_best, out_best_score, out_mapped, b_match=0.4, threshold=20.0,
                          stream=None):
    import torch
    n_chains = chain_gap_off.numel()
    n_reads = cand_off.numel()
    for t, nm, k in ((chain_gap_cnt, "chain_gap_cnt", n_chains), (chain_events, "chain_events", n_chains),
                     (out_chain_cost, "out_chain_cost", n_chains), (cand_cnt, "cand_cnt", n_reads),
                     (out_best, "out_best", n_reads), (out_best_score, "out_best_score", n_reads),
                     (out_mapped, "out_mapped", n_reads)):
        if t.numel() != k:
            raise ValueError(f"{nm} has {t.numel()} elements, expected {k}")
    _check(load().rawalign_chain_decide(
        _dev(gap_cost, torch.float32, "gap_cost"), gap_cost.numel(),
        _dev(chain_gap_off, torch.int64, "chain_gap_off"), _dev(chain_gap_cnt, torch.int32, "chain_gap_cnt"),
        _dev(chain_events, torch.int32, "chain_events"), n_chains,
        _dev(cand_off, torch.int64, "cand_off"), _dev(cand_cnt, torch.int32, "cand_cnt"), n_reads,
        float(b_match), float(threshold), _dev(out_chain_cost, torch.float32, "out_chain_cost"),
        _dev(out_best, torch.int32, "out_best"), _dev(out_best_score, torch.float64, "out_best_score"),
        _dev(out_mapped, torch.uint8, "out_mapped"), _stream(stream)))


def rawalign_autotune(q, q_off, q_len, r, r_off, r_len, out_score, out_end, cache_path=None, stream=None) -> Opts:
    best = Opts()
    _check(load().rawalign_autotune(*_pair_args(q, q_off, q_len, r, r_off, r_len, out_score, out_end),
                                    _stream(stream), None if cache_path is None else cache_path.encode(),
                                    ctypes.byref(best)))
    return best


def rawalign_load_tuning(cache_path: str) -> Opts:
    o = Opts()
    _check(load().rawalign_load_tuning(cache_path.encode(), ctypes.byref(o)))
    return o


def rawalign_last_timing() -> Timing:
    t = Timing()
    _check(load().rawalign_last_timing(ctypes.byref(t)))
    return t


def rawalign_version() -> str:
    return load().rawalign_version().decode()


# ---- convenience: packed batches on the device --------------------------------

class DeviceBatch:
    """A workloads.Batch copied to device tensors, plus output buffers."""

    def __init__(self, batch, device="cuda"):
        import torch
        self.batch = batch
        self.q = torch.from_numpy(np.ascontiguousarray(batch.q)).to(device)
        self.r = torch.from_numpy(np.ascontiguousarray(batch.r)).to(device)
        self.q_off = torch.from_numpy(batch.q_off.astype(np.int64)).to(device)
        self.q_len = torch.from_numpy(batch.q_len.astype(np.int32)).to(device)
        self.r_off = torch.from_numpy(batch.r_off.astype(np.int64)).to(device)
        self.r_len = torch.from_numpy(batch.r_len.astype(np.int32)).to(device)
        n = batch.n_pairs
        self.score = torch.empty(n, dtype=torch.float32, device=device)
        self.end = torch.empty(n, dtype=torch.int32, device=device)

    def args(self):
        return (self.q, self.q_off, self.q_len, self.r, self.r_off, self.r_len, self.score, self.end)

    def run(self, opts=None, plain=False, stream=None):
        if plain:
            rawalign_dtw_batch(*self.args(), stream=stream)
        else:
            rawalign_dtw_batch_ex(*self.args(), opts=opts, stream=stream)

    def results(self):
        import torch
        torch.cuda.synchronize()
        return self.score.cpu().numpy(), self.end.cpu().numpy()


class DeviceAnchored:
    """A workloads.AnchoredBatch on the device: gap DTW (rawalign_dtw_global_batch)
    then chain sums and the decision (rawalign_chain_decide)."""

    def __init__(self, ab, device="cuda"):
        import torch

        def t(x, dt):
            return torch.from_numpy(np.ascontiguousarray(x).astype(dt)).to(device)

        self.ab = ab
        self.q = t(ab.q, np.float32)
        self.r = t(ab.r, np.float32)
        self.gap_q_off, self.gap_q_len = t(ab.gap_q_off, np.int64), t(ab.gap_q_len, np.int32)
        self.gap_r_off, self.gap_r_len = t(ab.gap_r_off, np.int64), t(ab.gap_r_len, np.int32)
        self.chain_gap_off, self.chain_gap_cnt = t(ab.chain_gap_off, np.int64), t(ab.chain_gap_cnt, np.int32)
        self.chain_events = t(ab.chain_events, np.int32)
        self.cand_off, self.cand_cnt = t(ab.cand_off, np.int64), t(ab.cand_cnt, np.int32)
        self.gap_cost = torch.empty(ab.n_gaps, dtype=torch.float32, device=device)
        self.gap_end = torch.empty(ab.n_gaps, dtype=torch.int32, device=device)
        self.chain_cost = torch.empty(ab.n_chains, dtype=torch.float32, device=device)
        n_reads = len(ab.cand_off)
        self.best = torch.empty(n_reads, dtype=torch.int32, device=device)
        self.best_score = torch.empty(n_reads, dtype=torch.float64, device=device)
        self.mapped = torch.empty(n_reads, dtype=torch.uint8, device=device)

    def run(self, opts=None, b_match=0.4, threshold=20.0, stream=None, ends=False):
        rawalign_dtw_global_batch(self.q, self.gap_q_off, self.gap_q_len, self.r, self.gap_r_off, self.gap_r_len,
                                  self.gap_cost, self.gap_end if ends else None, opts=opts, stream=stream)
        rawalign_chain_decide(self.gap_cost, self.chain_gap_off, self.chain_gap_cnt, self.chain_events,
                              self.cand_off, self.cand_cnt, self.chain_cost, self.best, self.best_score,
                              self.mapped, b_match=b_match, threshold=threshold, stream=stream)

    def results(self):
        import torch
        torch.cuda.synchronize()
        return (self.gap_cost.cpu().numpy(), self.chain_cost.cpu().numpy(), self.best.cpu().numpy(),
                self.best_score.cpu().numpy(), self.mapped.cpu().numpy())


def dtw(batch, opts=None, plain=False):
    """Align a workloads.Batch on the GPU -> (scores float32, ends int32) on the host."""
    db = DeviceBatch(batch)
    db.run(opts=opts, plain=plain)
    return db.results()
