"""GPU parity: librawalign (HIP, gfx950) against the CPU oracle, through the C ABI."""
import math

import numpy as np
import pytest

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


def _say(msg):
    print(msg, flush=True)


def _run(L, b, **kw):
    plain = kw.pop("plain", False)
    opts = L.make_opts(**kw) if kw else None
    _say(f"  gpu: {b.name} pairs={b.n_pairs} max_n={int(b.q_len.max()) if b.n_pairs else 0} "
         f"max_m={int(b.r_len.max()) if b.n_pairs else 0} plain={plain} opts={kw}")
    db = L.DeviceBatch(b)
    db.run(opts=opts, plain=plain)
    return db.results()


def test_single_read(L):
    b = W.single_read()
    s, e = _run(L, b)
    st = parity.check(b, s, e)
    print("single_read", st)
    ps, pe = _run(L, b, plain=True)
    assert np.array_equal(s.view(np.uint32), ps.view(np.uint32)) and np.array_equal(e, pe)
    # the true candidate (pair 0) ends inside the read's source window
    assert int(np.argmin(s)) == 0


@pytest.mark.parametrize("seed", [0, 1])
def test_random_shapes_every_column_class(L, seed):
    """Region lengths around every columns-per-lane boundary (multiples of
    256), query lengths from 1 to above the 64-lane skew."""
    rng = np.random.default_rng(100 + seed)
    ms = []
    for k in range(1, 17):
        ms += [256 * k - 1, 256 * k, 256 * k + 1 if k < 16 else 4096]
    ms += [1, 2, 3, 63, 64, 65, 127, 128, 129]
    ns = rng.integers(1, 200, size=len(ms))
    ns[:6] = [1, 2, 63, 64, 65, 130]
    reads = [rng.standard_normal(int(n)).astype(np.float32) for n in ns]
    r = rng.standard_normal(int(sum(ms)) + 7).astype(np.float32)
    pairs, off = [], 3
    for i, m in enumerate(ms):
        pairs.append((i, off, int(m), False))
        off += int(m)
    b = W._pack("shapes", reads, pairs, r, {})
    s, e = _run(L, b)
    st = parity.check(b, s, e)
    print("shapes", st)


def test_degenerate_and_invalid_pairs(L):
    import torch
    rng = np.random.default_rng(7)
    q = rng.standard_normal(50).astype(np.float32)
    r = rng.standard_normal(80).astype(np.float32)
    # (q_off, q_len, r_off, r_len) -> expected sentinel or oracle
    rows = [(0, 0, 0, 10, (0.0, -1)),          # empty query
            (0, 5, 0, 0, (math.inf, -1)),      # empty region
            (0, 0, 0, 0, (0.0, -1)),           # both empty
            (45, 10, 0, 10, "nan"),            # query slice past the end
            (0, 5, 75, 10, "nan"),             # region slice past the end
            (-1, 5, 0, 10, "nan"),             # negative offset
            (0, -3, 0, 10, "nan"),             # negative length
            (0, 5, 0, 70000, "nan"),           # region above the maximum
            (0, 50, 0, 80, None),              # a normal pair in between
            (10, 1, 5, 1, None)]
    dev = "cuda"
    q_off = torch.tensor([x[0] for x in rows], dtype=torch.int64, device=dev)
    q_len = torch.tensor([x[1] for x in rows], dtype=torch.int32, device=dev)
    r_off = torch.tensor([x[2] for x in rows], dtype=torch.int64, device=dev)
    r_len = torch.tensor([x[3] for x in rows], dtype=torch.int32, device=dev)
    qt = torch.from_numpy(q).to(dev)
    rt = torch.from_numpy(r).to(dev)
    for plain in (False, True):
        sc = torch.full((len(rows),), -7.0, device=dev)
        en = torch.full((len(rows),), -7, dtype=torch.int32, device=dev)
        if plain:
            L.rawalign_dtw_batch(qt, q_off, q_len, rt, r_off, r_len, sc, en)
        else:
            L.rawalign_dtw_batch_ex(qt, q_off, q_len, rt, r_off, r_len, sc, en)
        torch.cuda.synchronize()
        sc, en = sc.cpu().numpy(), en.cpu().numpy()
        for i, row in enumerate(rows):
            exp = row[4]
            if exp == "nan":
                assert math.isnan(sc[i]) and en[i] == -2, (i, sc[i], en[i])
            elif exp is None:
                qq = q[row[0]:row[0] + row[1]]
                rr = r[row[2]:row[2] + row[3]]
                from oracle import oracle
                c32, e32 = oracle.dtw_f32(qq, rr)
                assert sc[i] == c32 and en[i] == e32
            else:
                assert sc[i] == exp[0] and en[i] == exp[1], (i, sc[i], en[i])


def test_plain_batch_full(L):
    b = W.plain_batch()
    s, e = _run(L, b)
    st = parity.check(b, s, e)
    print("plain_batch", st)
    ps, pe = _run(L, b, plain=True)
    assert np.array_equal(s.view(np.uint32), ps.view(np.uint32)) and np.array_equal(e, pe)


def test_long_regions_multi_stripe(L):
    """Regions above one stripe's 4096 columns are swept stripe by stripe by
    one wave; every launch setting gives bit-identical results."""
    rng = np.random.default_rng(3)
    ms = [4097, 5000, 8191, 8192, 8193, 12000, 16384, 16385, 20000, 24576, 30000, 32768, 40000, 65536]
    ns = [1, 2, 64, 65, 97, 200, 33, 130, 250, 7, 100, 64, 16384, 70]
    reads = [rng.standard_normal(n).astype(np.float32) for n in ns]
    r = rng.standard_normal(sum(ms)).astype(np.float32)
    pairs, off = [], 0
    for i, m in enumerate(ms):
        pairs.append((i, off, m, False))
        off += m
    b = W._pack("long", reads, pairs, r, {})
    s, e = _run(L, b)
    st = parity.check(b, s, e)
    print("long", st)
    for kw in ({"streams": 3}, {"long_waves_per_cu": 2}, {"plain": True}, {"long_kernel": L.LONG_ANTIDIAG},
               {"long_kernel": L.LONG_ANTIDIAG, "mode": L.MODE_PLAIN}):
        s2, e2 = _run(L, b, **kw)
        assert np.array_equal(s.view(np.uint32), s2.view(np.uint32)) and np.array_equal(e, e2), kw


def test_antidiag_kernel_against_oracle(L):
    """The anti-diagonal kernel on its own: queries around its row-block
    sizes (256 threads x 2 to 8 rows, picked per pair by a step-count
    model) and several blocks, regions just above one stripe up to the
    maximum, against the float oracle bit for bit."""
    from oracle import oracle
    rng = np.random.default_rng(5)
    ns = [1, 2, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049, 4096, 4097, 8193, 16384, 3, 700]
    ms = [4097, 4098, 5000, 4097, 9000, 4500, 4200, 6000, 4300, 4100, 5000, 4500, 4200, 7000, 4500, 4200, 4300,
          4100, 65536, 20000]
    reads = [rng.standard_normal(n).astype(np.float32) for n in ns]
    r = rng.standard_normal(sum(ms)).astype(np.float32)
    pairs, off = [], 0
    for i, m in enumerate(ms):
        pairs.append((i, off, m, False))
        off += m
    b = W._pack("antidiag", reads, pairs, r, {})
    s, e = _run(L, b, long_kernel=L.LONG_ANTIDIAG)
    for p in range(b.n_pairs):
        q = b.q[b.q_off[p]:b.q_off[p] + b.q_len[p]]
        rr = b.r[b.r_off[p]:b.r_off[p] + b.r_len[p]]
        c32, e32 = oracle.dtw_f32(q, rr)
        assert s[p].view(np.uint32) == np.float32(c32).view(np.uint32) and e[p] == e32, p
    parity.check(b, s, e)


def test_antidiag_short_regions_padded_stride(L):
    """With the single-stripe cut-off at 2,048 levels the anti-diagonal
    kernel takes regions of 2,049 levels up, whose 257..383 column tiles
    are padded to a 384-tile row-block stride; queries span one to many
    row blocks of every row count.  Equal to the oracle bit for bit and to
    the lane-striped kernel, in persistent and plain mode."""
    from oracle import oracle
    rng = np.random.default_rng(6)
    ns = [1, 5, 300, 511, 512, 513, 1100, 2049, 3000, 5000, 7, 640, 1537, 2048, 4097]
    ms = [2049, 2050, 2100, 2500, 3071, 3072, 3073, 2049, 3200, 2300, 4096, 4095, 2056, 2400, 2049]
    reads = [rng.standard_normal(n).astype(np.float32) for n in ns]
    r = rng.standard_normal(sum(ms)).astype(np.float32)
    pairs, off = [], 0
    for i, m in enumerate(ms):
        pairs.append((i, off, m, False))
        off += m
    b = W._pack("antidiag_short", reads, pairs, r, {})
    s, e = _run(L, b, long_kernel=L.LONG_ANTIDIAG, single_max=2048)
    for p in range(b.n_pairs):
        q = b.q[b.q_off[p]:b.q_off[p] + b.q_len[p]]
        rr = b.r[b.r_off[p]:b.r_off[p] + b.r_len[p]]
        c32, e32 = oracle.dtw_f32(q, rr)
        assert s[p].view(np.uint32) == np.float32(c32).view(np.uint32) and e[p] == e32, p
    s2, e2 = _run(L, b, long_kernel=L.LONG_ANTIDIAG, single_max=2048, mode=L.MODE_PLAIN)
    assert np.array_equal(s.view(np.uint32), s2.view(np.uint32)) and np.array_equal(e, e2)
    s3, e3 = _run(L, b, single_max=2048)
    assert np.array_equal(s.view(np.uint32), s3.view(np.uint32)) and np.array_equal(e, e3)


def test_antidiag_ties_first_column(L):
    """Small-integer queries and levels, so the last row holds the same
    minimum at many columns, within a tile and across tiles and row blocks.
    The shapes put row n-1 at the last row slot of its thread (no weight-0
    rows below it) and at an inner slot (weight-0 rows carry its prefix
    minimum down), on one and on several row blocks, for every rows-per-
    thread count the kernel's step-count model picks (2 to 8; it gives 2
    only to single-block pairs).  Regions of 2,049-4,096 levels run at the
    2,048-level cut-off.  Score bits and first column equal the float
    oracle's."""
    from oracle import oracle
    rng = np.random.default_rng(12)
    ns = [1, 2, 3, 255, 256, 511, 600, 601, 602, 603, 1023, 1024, 1500, 1501, 1502, 1503, 2047, 2048, 2049,
          2600, 2601, 2602, 2603, 2604, 2605, 2606, 2607, 3072, 4095, 4096, 4097, 5003, 6143, 6144]
    ms = [4097 + int(rng.integers(0, 5000)) for _ in ns]
    # shapes that complete the cases above (R picked: 5, 5, 7, 7, 4, 4, 5, 7; then 3, 3)
    ns += [1025, 1026, 1537, 1540, 1793, 1796, 2050, 3073, 1281, 1282]
    ms += [4097] * 8 + [3300, 3300]
    reads = [rng.integers(0, 3, n).astype(np.float32) for n in ns]
    r = rng.integers(0, 3, sum(ms)).astype(np.float32)
    pairs, off = [], 0
    for i, m in enumerate(ms):
        pairs.append((i, off, m, False))
        off += m
    b = W._pack("antidiag_ties", reads, pairs, r, {})
    for kw in (dict(long_kernel=L.LONG_ANTIDIAG), dict(long_kernel=L.LONG_ANTIDIAG, mode=L.MODE_PLAIN),
               dict(long_kernel=L.LONG_ANTIDIAG, single_max=2048)):
        print(f"  gpu: antidiag ties {kw}", flush=True)
        s, e = _run(L, b, **kw)
        for p in range(b.n_pairs):
            q = b.q[b.q_off[p]:b.q_off[p] + b.q_len[p]]
            rr = b.r[b.r_off[p]:b.r_off[p] + b.r_len[p]]
            c32, e32 = oracle.dtw_f32(q, rr)
            assert s[p].view(np.uint32) == np.float32(c32).view(np.uint32) and e[p] == e32, (p, ns[p], ms[p])


def test_antidiag_uneven_batch(L):
    """The 100,000-pair uneven batch with the anti-diagonal kernel on every
    region above one stripe (at both cut-offs) equals the default path."""
    b = W.uneven_batch()
    db = L.DeviceBatch(b)
    db.run(opts=L.make_opts())
    ref = [x.copy() for x in db.results()]
    for kw in (dict(long_kernel=L.LONG_ANTIDIAG), dict(long_kernel=L.LONG_ANTIDIAG, single_max=2048)):
        print(f"  gpu: uneven batch {kw}", flush=True)
        db.run(opts=L.make_opts(**kw))
        s, e = db.results()
        assert np.array_equal(s.view(np.uint32), ref[0].view(np.uint32)) and np.array_equal(e, ref[1]), kw


def test_long_stress_antidiag_equals_striped(L):
    """Full 1,024 x (10,000 x 20,000) batch: anti-diagonal and lane-striped
    kernels give the same bits."""
    b = W.long_stress()
    s, e = _run(L, b)
    s2, e2 = _run(L, b, long_kernel=L.LONG_ANTIDIAG)
    assert np.array_equal(s.view(np.uint32), s2.view(np.uint32)) and np.array_equal(e, e2)


def test_long_query_limit(L):
    """A multi-stripe pair above the long-query limit gets the sentinel; a
    single-stripe pair with the same query does not."""
    rng = np.random.default_rng(4)
    n = L.RAWALIGN_MAX_QUERY_LONG + 1
    reads = [rng.standard_normal(n).astype(np.float32)]
    r = rng.standard_normal(5000).astype(np.float32)
    b = W._pack("limit", reads, [(0, 0, 4097, False), (0, 0, 300, False)], r, {})
    s, e = _run(L, b)
    assert math.isnan(s[0]) and e[0] == -2
    parity.check(b, s, e, pairs=[1])


def test_long_stress_sampled(L):
    """Full 1,024 x (10,000 x 20,000) batch on the GPU, 16 pairs against the
    oracle."""
    b = W.long_stress()
    s, e = _run(L, b)
    sample = np.arange(0, b.n_pairs, b.n_pairs // 16)[:16]
    st = parity.check(b, s, e, pairs=sample)
    print("long_stress", st)
    assert np.isfinite(s).all() and (e >= 0).all() and (e < b.r_len).all()


def test_uneven_batch_persistent_vs_plain_and_sample(L):
    """Full 100,000-pair uneven batch: persistent (default and autotuned, the
    setting the benchmark times) and plain bit-identical, and a stratified
    sample of 200 pairs against the oracle."""
    b = W.uneven_batch()
    db = L.DeviceBatch(b)
    _say(f"  gpu: {b.name} persistent")
    db.run(opts=L.make_opts())
    s, e = db.results()
    _say(f"  gpu: {b.name} plain")
    db.run(plain=True)
    ps, pe = db.results()
    assert np.array_equal(s.view(np.uint32), ps.view(np.uint32)) and np.array_equal(e, pe)
    _say(f"  gpu: {b.name} autotune")
    best = L.rawalign_autotune(*db.args())
    db.score.fill_(-1.0)
    db.run(opts=best)
    ts, te = db.results()
    assert np.array_equal(s.view(np.uint32), ts.view(np.uint32)) and np.array_equal(e, te), best.as_dict()
    sample = parity.stratified_sample(b, 200)
    st = parity.check(b, s, e, pairs=sample)
    print("uneven_batch", st)
    assert np.isfinite(s).all() and (e >= 0).all() and (e < b.r_len).all()


def test_exact_inputs_match_double(L):
    """Quarter-integer inputs keep every sum exact in float, so the GPU must
    equal the double oracle exactly, designed ties included."""
    rng = np.random.default_rng(9)
    b = W.random_pairs(rng, 300, (1, 300), (1, 5000), value_fn=lambda g, n: W.dyadic_values(g, n, -2, 2, 0.5))
    s, e = _run(L, b)
    s64, e64, _, _ = parity.oracle_batch(b)
    assert np.array_equal(s.astype(np.float64), s64) and np.array_equal(e, e64)


def test_decide_matches_oracle(L):
    import torch
    from oracle import oracle
    b = W.plain_batch(n_pairs=600)
    s32, _, _ = oracle.dtw_batch_f32(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, parity.threads())
    s32 = s32.copy()
    s32[5] = np.inf  # a candidate with an empty region
    # NaN sentinels (pairs that were not aligned) are no candidates: one
    # before a read's other candidates, and a read with nothing else
    s32[int(b.cand_off[1])] = np.nan
    s32[int(b.cand_off[2]):int(b.cand_off[2] + b.cand_cnt[2])] = np.nan
    dev = "cuda"
    n_reads = len(b.cand_off)
    ob = torch.empty(n_reads, dtype=torch.int32, device=dev)
    os_ = torch.empty(n_reads, dtype=torch.float64, device=dev)
    om = torch.empty(n_reads, dtype=torch.uint8, device=dev)
    cnt = b.cand_cnt.copy()
    cnt[3] = 0  # a read without candidates
    for bm, th in ((0.4, 20.0), (0.3, 5.0)):
        _say(f"  gpu: decide reads={n_reads} b_match={bm} threshold={th}")
        L.rawalign_decide(torch.from_numpy(s32).to(dev), torch.from_numpy(b.cand_off).to(dev),
                          torch.from_numpy(cnt).to(dev), torch.from_numpy(b.n_events).to(dev),
                          ob, os_, om, b_match=bm, threshold=th)
        torch.cuda.synchronize()
        rb, rs, rm = oracle.decide(s32, b.cand_off, cnt, b.n_events, bm, th)
        assert rb[1] > b.cand_off[1] and rb[2] == -1 and rs[2] == -np.inf
        assert np.array_equal(ob.cpu().numpy(), rb)
        assert np.array_equal(os_.cpu().numpy(), rs)
        assert np.array_equal(om.cpu().numpy(), rm)


def test_decide_ties_and_many_candidates(L):
    """The decision of a read spread over a wave's lanes: costs drawn from a
    few values, so that equal best scores fall on candidates of different
    lanes and of the same lane, NaN sentinels and +inf costs among them, and
    reads of 0 to 300 candidates (one and several candidates per lane).  The
    best index, score and flag equal the oracle's first-highest scan."""
    import torch
    from oracle import oracle
    rng = np.random.default_rng(41)
    counts = np.array([0, 1, 2, 63, 64, 65, 127, 128, 129, 200, 300, 5, 64, 130] * 6, dtype=np.int32)
    n_reads = len(counts)
    cand_off = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    n_pairs = int(counts.sum())
    cost = rng.choice(np.array([0.5, 1.0, 2.0, 3.0, np.inf, np.nan], dtype=np.float32), size=n_pairs,
                      p=[0.1, 0.2, 0.3, 0.2, 0.1, 0.1]).astype(np.float32)
    # reads whose candidates are all +inf, all NaN, or tie at one value everywhere
    for k, v in ((1, np.inf), (2, np.nan), (3, 2.0), (4, 1.0)):
        cost[cand_off[k]:cand_off[k] + counts[k]] = v
    n_events = rng.integers(0, 120, size=n_reads).astype(np.int32)
    dev = "cuda"
    ob = torch.empty(n_reads, dtype=torch.int32, device=dev)
    os_ = torch.empty(n_reads, dtype=torch.float64, device=dev)
    om = torch.empty(n_reads, dtype=torch.uint8, device=dev)
    for bm, th in ((0.4, 20.0), (0.0, 0.0), (0.3, -1.0)):
        _say(f"  gpu: decide ties reads={n_reads} pairs={n_pairs} b_match={bm}")
        L.rawalign_decide(torch.from_numpy(cost).to(dev), torch.from_numpy(cand_off).to(dev),
                          torch.from_numpy(counts).to(dev), torch.from_numpy(n_events).to(dev),
                          ob, os_, om, b_match=bm, threshold=th)
        torch.cuda.synchronize()
        rb, rs, rm = oracle.decide(cost, cand_off, counts, n_events, bm, th)
        assert np.array_equal(ob.cpu().numpy(), rb)
        assert np.array_equal(os_.cpu().numpy().view(np.uint64), rs.view(np.uint64))
        assert np.array_equal(om.cpu().numpy(), rm)
    # the ties really occur: several reads have more than one best candidate
    # in different lanes (indices 64 or more apart)
    multi = 0
    for k in range(n_reads):
        c = cost[cand_off[k]:cand_off[k] + counts[k]].astype(np.float64)
        ok = ~np.isnan(c)
        if ok.sum() < 2:
            continue
        best = np.flatnonzero(ok & (c == np.nanmin(c)))
        multi += int(best.max() - best.min() >= 64)
    assert multi >= 10


def test_autotune_and_tuning_cache(L, tmp_path):
    """The autotuner picks a valid setting, writes it to a cache that loads
    back to the same setting, and the tuned path (opts NULL) gives the same
    bits as the defaults."""
    b = W.plain_batch(n_pairs=1500)
    db = L.DeviceBatch(b)
    _say(f"  gpu: autotune {b.name} pairs={b.n_pairs}")
    db.run(opts=L.make_opts())
    s0, e0 = db.results()
    cache = str(tmp_path / "tune.json")
    best = L.rawalign_autotune(*db.args(), cache_path=cache)
    assert best.mode == L.MODE_PERSISTENT and best.streams in (1, 3)
    loaded = L.rawalign_load_tuning(cache)
    assert loaded.as_dict() == best.as_dict()
    db.score.fill_(-1.0)
    db.run()   # opts NULL: the tuned setting
    s1, e1 = db.results()
    assert np.array_equal(s0.view(np.uint32), s1.view(np.uint32)) and np.array_equal(e0, e1)


def test_tuned_antidiag_setting(L, tmp_path):
    """A tuned setting that names the anti-diagonal kernel (a tuning cache
    edited to it) runs plain batches with that kernel (opts NULL equals the
    explicit setting and the striped kernel), while the alignment-start
    entry point, inheriting it with opts NULL, takes the striped kernel
    instead of failing; explicit anti-diagonal opts are still rejected
    there.  The device's tuned setting is put back to the defaults after."""
    import json
    import torch
    rng = np.random.default_rng(21)
    ns, ms = [300, 2600, 700, 5000], [5000, 9000, 4500, 4200]
    reads = [rng.standard_normal(n).astype(np.float32) for n in ns]
    r = rng.standard_normal(sum(ms)).astype(np.float32)
    pairs, off = [], 0
    for i, m in enumerate(ms):
        pairs.append((i, off, m, False))
        off += m
    b = W._pack("tuned_antidiag", reads, pairs, r, {})
    db = L.DeviceBatch(b)
    _say(f"  gpu: tuned anti-diagonal setting pairs={b.n_pairs}")
    cache = str(tmp_path / "tune.json")
    L.rawalign_autotune(*db.args(), cache_path=cache)   # a cache for this device and library version
    doc = json.load(open(cache))

    def load_with(**fields):
        d = dict(doc, **fields)
        path = str(tmp_path / "edited.json")
        json.dump(d, open(path, "w"))
        return L.rawalign_load_tuning(path)

    start = torch.empty(b.n_pairs, dtype=torch.int32, device="cuda")

    def span(opts):
        L.rawalign_dtw_span(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, db.score, db.end, start,
                            opts=opts)
        torch.cuda.synchronize()
        return db.score.cpu().numpy(), db.end.cpu().numpy(), start.cpu().numpy()

    try:
        db.run(opts=L.make_opts())
        s0, e0 = db.results()
        sp0 = span(L.make_opts())
        loaded = load_with(long_kernel=L.LONG_ANTIDIAG, long_waves_per_cu=0, pipe_waves=0)
        assert loaded.long_kernel == L.LONG_ANTIDIAG
        db.run()   # opts NULL: the tuned anti-diagonal setting
        s1, e1 = db.results()
        db.run(opts=L.make_opts(long_kernel=L.LONG_ANTIDIAG, single_max=int(doc["single_max"])))
        s2, e2 = db.results()
        for s, e in ((s1, e1), (s2, e2)):
            assert np.array_equal(s0.view(np.uint32), s.view(np.uint32)) and np.array_equal(e0, e)
        sp1 = span(None)   # inherits the setting: striped kernel
        for x, y in zip(sp0, sp1):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
        with pytest.raises(L.RawAlignError):
            span(L.make_opts(long_kernel=L.LONG_ANTIDIAG))
    finally:
        d = L.opts_default().as_dict()
        load_with(**{k: v for k, v in d.items() if k != "flags"})


def test_million_event_query_and_64bit_offsets(L):
    """A single-stripe pair with a query of a million events, and pairs whose
    query and region slices start beyond 2^31 elements (8 GiB arrays), against
    the float oracle bit for bit."""
    import torch
    from oracle import oracle
    rng = np.random.default_rng(11)
    dev = "cuda"
    big = (1 << 31) + 4096
    q_long = rng.standard_normal(1_000_003).astype(np.float32)
    r_small = rng.standard_normal(100).astype(np.float32)
    q_hi = rng.standard_normal(300).astype(np.float32)
    r_hi = rng.standard_normal(5000).astype(np.float32)
    _say("  gpu: 8 GiB query and region arrays for 64-bit offsets")
    q = torch.zeros(big, dtype=torch.float32, device=dev)
    r = torch.zeros(big, dtype=torch.float32, device=dev)
    q[:len(q_long)] = torch.from_numpy(q_long).to(dev)
    r[:len(r_small)] = torch.from_numpy(r_small).to(dev)
    qo, ro = (1 << 31) + 7, (1 << 31) - 1000   # the region straddles 2^31
    q[qo:qo + len(q_hi)] = torch.from_numpy(q_hi).to(dev)
    r[ro:ro + len(r_hi)] = torch.from_numpy(r_hi).to(dev)
    rows = [(0, len(q_long), 0, len(r_small)), (qo, len(q_hi), ro, len(r_hi)), (qo, len(q_hi), ro, 1500)]
    t = lambda xs, dt: torch.tensor(xs, dtype=dt, device=dev)
    q_off = t([x[0] for x in rows], torch.int64)
    q_len = t([x[1] for x in rows], torch.int32)
    r_off = t([x[2] for x in rows], torch.int64)
    r_len = t([x[3] for x in rows], torch.int32)
    sc = torch.empty(len(rows), dtype=torch.float32, device=dev)
    en = torch.empty(len(rows), dtype=torch.int32, device=dev)
    L.rawalign_dtw_batch_ex(q, q_off, q_len, r, r_off, r_len, sc, en)
    torch.cuda.synchronize()
    s, e = sc.cpu().numpy(), en.cpu().numpy()
    del q, r
    torch.cuda.empty_cache()
    refs = [(q_long, r_small), (q_hi, r_hi), (q_hi, r_hi[:1500])]
    for i, (qq, rr) in enumerate(refs):
        c32, e32 = oracle.dtw_f32(qq, rr)
        assert s[i].view(np.uint32) == np.float32(c32).view(np.uint32) and e[i] == e32, i
