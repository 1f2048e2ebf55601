"""GPU parity of the warping path (rawalign_dtw_path, Sec. 2.4: the
alignment path as an optional output) through the C ABI: score, end, start
and every read event's level range bit for bit against the float oracle over
interval widths in every columns-per-lane class, exact against the double
oracle on dyadic inputs (where ties are frequent, so the tie order is
exercised), the sentinels, and pairs of the single read and the uneven
batch."""
import numpy as np
import pytest

from oracle import oracle
from paper_2310_05037_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_2310_05037_amd import lib
    assert torch.cuda.is_available()
    lib.load()
    return lib


def _gpu_path(L, b, max_query, path_off=None, path_size=None):
    import torch
    print(f"  gpu: path {b.name} pairs={b.n_pairs} max_n={int(b.q_len.max()) if b.n_pairs else 0} "
          f"max_m={int(b.r_len.max()) if b.n_pairs else 0} max_query={max_query}", flush=True)
    db = L.DeviceBatch(b)
    n = b.n_pairs
    rows = np.maximum(b.q_len.astype(np.int64), 0)
    if path_off is None:
        path_off = np.concatenate([[0], np.cumsum(rows)[:-1]]).astype(np.int64)
    if path_size is None:
        path_size = int(rows.sum())
    lo = torch.full((path_size,), -7, dtype=torch.int32, device="cuda")
    hi = torch.full((path_size,), -7, dtype=torch.int32, device="cuda")
    start = torch.empty(n, dtype=torch.int32, device="cuda")
    L.rawalign_dtw_path(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, max_query,
                        torch.from_numpy(path_off).cuda(), lo, hi, db.score, db.end, start)
    torch.cuda.synchronize()
    return (db.score.cpu().numpy(), db.end.cpu().numpy(), start.cpu().numpy(), lo.cpu().numpy(),
            hi.cpu().numpy(), path_off)


def _check(b, res, pairs, exact64=False):
    s, e, st, lo, hi, off = res
    for p in pairs:
        n = int(b.q_len[p])
        q = b.q[b.q_off[p]:b.q_off[p] + n]
        r = b.r[b.r_off[p]:b.r_off[p] + int(b.r_len[p])]
        c, oe, ost, g, olo, ohi = (oracle.dtw_path_f64 if exact64 else oracle.dtw_path_f32)(q, r)
        ctx = (int(p), n, int(b.r_len[p]), oe, ost)
        if exact64:
            assert float(s[p]) == c, ctx
        else:
            assert s[p].view(np.uint32) == np.float32(c).view(np.uint32), ctx
        assert e[p] == oe and st[p] == ost, (ctx, int(e[p]), int(st[p]))
        got_lo, got_hi = lo[off[p]:off[p] + n], hi[off[p]:off[p] + n]
        bad = np.flatnonzero((got_lo != olo) | (got_hi != ohi))
        assert len(bad) == 0, (ctx, [(int(i), int(got_lo[i]), int(olo[i]), int(got_hi[i]), int(ohi[i]))
                                     for i in bad[:5]])


def _embedded(rng, spans, name, noise=0.1, dwell_p=0.35, value_fn=None):
    """One pair per span: the query follows `span` consecutive levels of its
    region with geometric dwell and noise, so the alignment covers about
    that many levels."""
    reads, pairs, chunks, off = [], [], [], 0
    for k, sp in enumerate(spans):
        m = sp + int(rng.integers(0, 200))
        r = value_fn(rng, m) if value_fn else rng.standard_normal(m).astype(np.float32)
        a = int(rng.integers(0, m - sp + 1))
        dw = rng.geometric(dwell_p, sp)
        q = np.repeat(r[a:a + sp], dw)
        if value_fn is None:
            q = q + rng.normal(0, noise, len(q))
        reads.append(q.astype(np.float32))
        chunks.append(r)
        pairs.append((k, off, m, True))
        off += m
    return W._pack(name, reads, pairs, np.concatenate(chunks).astype(np.float32), {})


def test_path_interval_widths(L):
    """Intervals from 1 to 2048 levels (every columns-per-lane class, lane
    and class boundaries), plus unrelated random pairs."""
    rng = np.random.default_rng(900)
    spans = [1, 2, 3, 63, 64, 65, 127, 128, 129, 200, 255, 256, 257, 400, 511, 512, 513, 700, 1000, 1300,
             1600, 1900, 2000]
    b = _embedded(rng, spans, "path_widths")
    res = _gpu_path(L, b, max_query=int(b.q_len.max()))
    s, e, st, lo, hi, off = res
    ok = np.flatnonzero(e - st + 1 <= 2048)
    assert len(ok) >= len(spans) - 2
    _check(b, res, ok)
    b2 = W.random_pairs(rng, 60, (1, 500), (1, 900))
    _check(b2, _gpu_path(L, b2, max_query=500), range(b2.n_pairs))


def test_path_exact_on_dyadic_inputs(L):
    """Quarter-step levels and exact copies: every sum is exact in float, so
    the paths equal the double oracle's, ties and all."""
    rng = np.random.default_rng(901)
    fn = lambda g, k: W.dyadic_values(g, k, -2.0, 2.0, 0.25)
    b = _embedded(rng, [5, 40, 64, 130, 300, 600, 1024], "path_dyadic", value_fn=fn)
    _check(b, _gpu_path(L, b, max_query=int(b.q_len.max())), range(b.n_pairs), exact64=True)
    b2 = W.random_pairs(rng, 80, (1, 120), (1, 160), value_fn=fn)
    _check(b2, _gpu_path(L, b2, max_query=120), range(b2.n_pairs), exact64=True)


def test_path_sentinels(L):
    """-4: more events than max_query, or an interval wider than 2048
    levels; -1: empty region; -2: invalid slice; an empty query has no
    entries; a pair whose entries leave the path arrays is not written."""
    rng = np.random.default_rng(902)
    b = _embedded(rng, [2600, 50, 50, 50, 50, 50], "path_sentinels")
    r_len = b.r_len.copy()
    q_len = b.q_len.copy()
    q_off = b.q_off.copy()
    r_len[2] = 0
    q_off[3] = len(b.q)
    q_len[4] = 0
    b = W.Batch(b.name, b.q, b.r, q_off, q_len, b.r_off, r_len, b.cand_off, b.cand_cnt, b.n_events,
                b.true_pair, b.meta)
    max_query = int(b.q_len[1]) - 1          # pair 1 exceeds it
    rows = np.maximum(b.q_len.astype(np.int64), 0)
    off = np.concatenate([[0], np.cumsum(rows)[:-1]]).astype(np.int64)
    size = int(rows.sum())
    off[5] = size - 3                           # pair 5 would run past the end
    s, e, st, lo, hi, off = _gpu_path(L, b, max_query, off, size)
    span = lambda p: slice(off[p], off[p] + int(b.q_len[p]))
    assert (lo[span(0)] == -4).all() and (hi[span(0)] == -4).all() and e[0] - st[0] + 1 > 2048
    assert (lo[span(1)] == -4).all() and (hi[span(1)] == -4).all()
    assert e[2] == -1 and (lo[span(2)] == -1).all() and (hi[span(2)] == -1).all()
    assert e[3] == -2 and (lo[span(3)] == -2).all() and (hi[span(3)] == -2).all()
    assert e[4] == -1 and st[4] == -1
    assert (lo[size - 3:] == -7).all() and (hi[size - 3:] == -7).all()


def test_path_single_read_and_uneven_batch_sample(L):
    """The single read's 10 candidates, and 40 pairs of the 100,000-pair
    uneven batch (intervals up to 2048 levels), bit for bit."""
    b = W.single_read()
    _check(b, _gpu_path(L, b, max_query=int(b.q_len.max())), range(b.n_pairs))
    u = W.uneven_batch()
    rng = np.random.default_rng(903)
    pick = np.sort(rng.choice(u.n_pairs, size=40, replace=False))
    sub = u.subset(pick)
    res = _gpu_path(L, sub, max_query=8000)
    s, e, st, lo, hi, off = res
    ok = np.flatnonzero((e >= 0) & (e - st + 1 <= 2048))
    assert len(ok) >= 30
    _check(sub, res, ok)
