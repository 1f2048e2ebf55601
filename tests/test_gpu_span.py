"""GPU parity of the alignment start (rawalign_dtw_span) through the C ABI:
score, end and start bit for bit against the float oracle on every route,
exact against the double oracle on dyadic inputs, and on sampled pairs of
the 100,000-pair uneven batch; the aligned interval's global cost equals
the score."""
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2310_05037_amd import workloads as W

from . import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_2310_05037_amd import lib
    assert torch.cuda.is_available()
    lib.load()
    return lib


def _gpu_span(L, b, **kw):
    import torch
    print(f"  gpu: span {b.name} pairs={b.n_pairs} max_n={int(b.q_len.max()) if b.n_pairs else 0} "
          f"max_m={int(b.r_len.max()) if b.n_pairs else 0} opts={kw}", flush=True)
    db = L.DeviceBatch(b)
    start = torch.empty(b.n_pairs, dtype=torch.int32, device="cuda")
    L.rawalign_dtw_span(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, db.score, db.end, start,
                        opts=L.make_opts(**kw) if kw else None)
    torch.cuda.synchronize()
    return db.score.cpu().numpy(), db.end.cpu().numpy(), start.cpu().numpy()


def _check_f32(b, s, e, st, pairs=None):
    sub = b if pairs is None else b.subset(pairs)
    s32, e32, st32 = oracle.dtw_span_batch_f32(sub.q, sub.q_off, sub.q_len, sub.r, sub.r_off, sub.r_len,
                                               parity.threads())
    if pairs is not None:
        s, e, st = s[pairs], e[pairs], st[pairs]
    assert np.array_equal(s.view(np.uint32), s32.view(np.uint32))
    assert np.array_equal(e, e32)
    bad = np.flatnonzero(st != st32)
    assert len(bad) == 0, [(int(p), int(st[p]), int(st32[p]), int(e[p])) for p in bad[:10]]
    return sub


def _check_interval(b, s, e, st, pairs):
    """The region interval [start, end] aligned globally costs C (double)."""
    for p in pairs:
        if e[p] < 0:
            continue
        q = b.q[b.q_off[p]:b.q_off[p] + b.q_len[p]]
        r = b.r[b.r_off[p] + st[p]:b.r_off[p] + e[p] + 1]
        g = oracle.dtw_global_f64(q, r)
        assert abs(g - float(s[p])) <= parity.REL_TOL * abs(g) + parity.ABS_TOL, (p, g, s[p])


@pytest.mark.parametrize("seed", [0, 1])
def test_span_every_route(L, seed):
    """Regions on every route (1 .. 6,000 levels, one and several stripes),
    queries from 1 event up; plain and persistent scheduling agree."""
    rng = np.random.default_rng(400 + seed)
    ms = [1, 2, 3, 63, 64, 65, 127, 128, 129, 700, 2047, 2048, 2049, 3000, 4096, 4097, 6000] * 3
    ns = rng.integers(1, 200, size=len(ms))
    ns[:4] = [1, 2, 63, 64]
    reads = [rng.standard_normal(int(n)).astype(np.float32) for n in ns]
    r = rng.standard_normal(int(sum(ms)) + 3).astype(np.float32)
    pairs, off = [], 0
    for k, m in enumerate(ms):
        pairs.append((k, off, int(m), False))
        off += int(m)
    b = W._pack(f"span_routes_{seed}", reads, pairs, r, {})
    s, e, st = _gpu_span(L, b)
    _check_f32(b, s, e, st)
    assert ((st >= 0) & (st <= e)).all()
    _check_interval(b, s, e, st, range(0, b.n_pairs, 5))
    s2, e2, st2 = _gpu_span(L, b, mode=L.MODE_PLAIN)
    assert np.array_equal(s.view(np.uint32), s2.view(np.uint32)) and np.array_equal(st, st2)


def test_span_exact_on_dyadic_inputs(L):
    """Quarter-integer values: every sum exact, so the double oracle's
    start (designed ties included) is the GPU's."""
    rng = np.random.default_rng(7)
    b = W.random_pairs(rng, 300, (1, 120), (1, 2500), value_fn=lambda g, k: W.dyadic_values(g, k, -2.0, 2.0, 0.5))
    s, e, st = _gpu_span(L, b)
    s64, e64, st64 = oracle.dtw_span_batch_f64(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, parity.threads())
    assert np.array_equal(s.astype(np.float64), s64) and np.array_equal(e, e64) and np.array_equal(st, st64)


def test_span_degenerate_and_invalid(L):
    rng = np.random.default_rng(8)
    b = W.random_pairs(rng, 60, (0, 50), (0, 80))
    q_len, r_len, q_off = b.q_len.copy(), b.r_len.copy(), b.q_off.copy()
    q_len[0], r_len[1] = 0, 0
    q_off[2], q_len[2] = len(b.q), 1      # slice past the end of q
    b = W.Batch(b.name, b.q, b.r, q_off, q_len, b.r_off, r_len, b.cand_off, b.cand_cnt, b.n_events,
                b.true_pair, b.meta)
    s, e, st = _gpu_span(L, b)
    assert s[0] == 0 and e[0] == -1 and st[0] == -1
    assert (q_len[1] == 0 or math.isinf(s[1])) and e[1] == -1 and st[1] == -1
    assert math.isnan(s[2]) and e[2] == -2 and st[2] == -2
    ok = np.ones(b.n_pairs, bool)
    ok[:3] = False
    _check_f32(b, s, e, st, np.flatnonzero(ok))


def test_span_uneven_batch_sampled(L):
    """The full 100,000-pair uneven batch, in the tuned persistent launch
    the benchmark uses; 150 stratified pairs against the oracle."""
    b = W.uneven_batch()
    s, e, st = _gpu_span(L, b)
    rng = np.random.default_rng(9)
    cells = b.q_len.astype(np.int64) * b.r_len.astype(np.int64)
    order = np.argsort(cells)
    pairs = np.sort(np.concatenate([order[-10:], rng.choice(order[:-10], 140, replace=False)]))
    _check_f32(b, s, e, st, pairs)
    _check_interval(b, s, e, st, pairs[::10])
    assert ((st >= 0) & (st <= e)).all()
