"""GPU parity of the pipelined multi-stripe kernel (RAWALIGN_LONG_PIPELINE,
waves of one workgroup sharing each pair) and of the single-stripe cut-off
(opts.single_max): every setting returns the bits of the single-wave
striped kernel and of the float oracle, through the C ABI."""
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


def _run(L, b, db=None, **kw):
    opts = L.make_opts(**kw)
    _say(f"  gpu: {b.name} pairs={b.n_pairs} max_n={int(b.q_len.max())} max_m={int(b.r_len.max())} opts={kw}")
    db = db or L.DeviceBatch(b)
    db.run(opts=opts)
    s, e = db.results()
    return s.copy(), e.copy()


def _same(x, y):
    return np.array_equal(x[0].view(np.uint32), y[0].view(np.uint32)) and np.array_equal(x[1], y[1])


def _long_pairs(seed, count, n_range, m_range):
    return W.random_pairs(np.random.default_rng(seed), count, n_range, m_range)


@pytest.mark.parametrize("waves", [2, 4, 8])
def test_pipeline_equals_striped_and_oracle(L, waves):
    """Regions of 2,049 to 40,000 levels (2 to 20 stripes: fewer, as many and
    more stripes than waves), queries from 1 event to past several hand-over
    blocks: the pipeline equals the single-wave kernel bit for bit and the
    float oracle, in persistent and plain mode."""
    b = _long_pairs(40 + waves, 160, (1, 700), (2049, 40000))
    db = L.DeviceBatch(b)
    ref = _run(L, b, db)
    got = _run(L, b, db, long_kernel=L.LONG_PIPELINE, pipe_waves=waves)
    assert _same(got, ref)
    print(parity.check(b, *got))
    plain = _run(L, b, db, long_kernel=L.LONG_PIPELINE, pipe_waves=waves, mode=L.MODE_PLAIN)
    assert _same(plain, ref)


def test_cutoff_2048_equals_4096(L):
    """Regions of 2,049 to 4,096 levels on two stripes (single_max 2048, both
    long kernels) or one (4096) give the same bits; queries longer than a
    stripe edge column keep one stripe either way."""
    b = _long_pairs(50, 300, (1, 900), (1900, 4300))
    db = L.DeviceBatch(b)
    ref = _run(L, b, db)
    for kw in (dict(single_max=2048), dict(single_max=2048, long_kernel=L.LONG_PIPELINE, pipe_waves=2),
               dict(single_max=2048, long_kernel=L.LONG_PIPELINE, pipe_waves=4)):
        assert _same(_run(L, b, db, **kw), ref), kw
    print(parity.check(b, *ref))
    # a query beyond RAWALIGN_MAX_QUERY_LONG against a 3,000-level region
    rng = np.random.default_rng(51)
    q = rng.standard_normal(L.RAWALIGN_MAX_QUERY_LONG + 100).astype(np.float32)
    r = rng.standard_normal(3000).astype(np.float32)
    lb = W._pack("long_query_3000", [q], [(0, 0, 3000, True)], r, {})
    a = _run(L, lb)
    c = _run(L, lb, single_max=2048, long_kernel=L.LONG_PIPELINE)
    assert _same(a, c) and np.isfinite(a[0][0]) and a[1][0] >= 0


def test_pipeline_long_stress(L):
    """The 1,024 x 10,000 x 20,000 batch: the pipeline at 2, 4 and 8 waves
    per pair equals the single-wave kernel on every pair."""
    b = W.long_stress()
    db = L.DeviceBatch(b)
    ref = _run(L, b, db)
    for waves in (2, 4, 8):
        assert _same(_run(L, b, db, long_kernel=L.LONG_PIPELINE, pipe_waves=waves), ref), waves


def test_pipeline_streaming_extension(L):
    """Resident rows on the pipeline (the corner of every stripe handed over
    before its left neighbour rewrites the row): chunk by chunk equals the
    whole prefix and the single-wave kernel, bit for bit, rows included."""
    import torch
    rng = np.random.default_rng(52)
    ms = np.array([4097, 6000, 9000, 20000, 2500, 12345], np.int32)
    n_jobs = len(ms)
    r = torch.from_numpy(rng.standard_normal(int(ms.sum())).astype(np.float32)).cuda()
    r_off = np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.int64)
    reads = [rng.standard_normal(int(rng.integers(150, 500))).astype(np.float32) for _ in range(n_jobs)]
    cuts = [sorted(rng.integers(1, len(x), size=2).tolist()) for x in reads]
    row_off = r_off.copy()
    results = {}
    for name, kw in (("striped", {}), ("pipe4", dict(long_kernel=L.LONG_PIPELINE, pipe_waves=4, single_max=2048))):
        rows = torch.zeros(int(ms.sum()), device="cuda")
        out = []
        for k in range(3):
            chunks = []
            for x, (c1, c2) in zip(reads, cuts):
                bounds = [0, c1, c2, len(x)]
                chunks.append(x[bounds[k]:bounds[k + 1]])
            q = np.concatenate(chunks)
            q_len = np.array([len(c) for c in chunks], np.int32)
            q_off = np.concatenate([[0], np.cumsum(q_len)[:-1]]).astype(np.int64)
            first = np.full(n_jobs, 1 if k == 0 else 0, np.uint8)
            score = torch.empty(n_jobs, device="cuda")
            end = torch.empty(n_jobs, dtype=torch.int32, device="cuda")
            _say(f"  gpu: extend {name} chunk {k}")
            L.rawalign_dtw_extend(torch.from_numpy(q).cuda(), torch.from_numpy(q_off).cuda(),
                                  torch.from_numpy(q_len).cuda(), r, torch.from_numpy(r_off).cuda(),
                                  torch.from_numpy(ms).cuda(), rows, torch.from_numpy(row_off).cuda(),
                                  torch.from_numpy(first).cuda(), score, end, opts=L.make_opts(**kw))
            torch.cuda.synchronize()
            out.append((score.cpu().numpy(), end.cpu().numpy()))
        results[name] = (out, rows.cpu().numpy())
    for k in range(3):
        assert _same(results["pipe4"][0][k], results["striped"][0][k]), k
    assert np.array_equal(results["pipe4"][1].view(np.uint32), results["striped"][1].view(np.uint32))
    # and the last chunk equals aligning each whole read at once
    from oracle import oracle
    for j in range(n_jobs):
        c, e = oracle.dtw_f32(reads[j], r[int(r_off[j]):int(r_off[j] + ms[j])].cpu().numpy())
        s, en = results["pipe4"][0][2][0][j], results["pipe4"][0][2][1][j]
        assert np.float32(c).view(np.uint32) == s.view(np.uint32) and e == en, j


def test_pipeline_uneven_batch(L):
    """The 100,000-pair uneven batch: pipeline and cut-off settings equal the
    default path on every pair."""
    b = W.uneven_batch()
    db = L.DeviceBatch(b)
    ref = _run(L, b, db)
    for kw in (dict(long_kernel=L.LONG_PIPELINE, pipe_waves=4),
               dict(long_kernel=L.LONG_PIPELINE, pipe_waves=2, single_max=2048)):
        assert _same(_run(L, b, db, **kw), ref), kw


def test_autotune_searches_shape_and_workgroup(L, tmp_path):
    """The autotuner over a batch with long regions returns a valid shape
    (cut-off, long kernel, waves per pair), the cache round-trips every
    field, and the tuned path (opts NULL) gives the defaults' bits."""
    b = _long_pairs(60, 400, (1, 600), (100, 20000))
    db = L.DeviceBatch(b)
    ref = _run(L, b, db)
    cache = str(tmp_path / "tune.json")
    _say(f"  gpu: autotune {b.name} pairs={b.n_pairs}")
    best = L.rawalign_autotune(*db.args(), cache_path=cache)
    print("tuned", best.as_dict())
    assert best.single_max in (2048, 4096)
    assert best.long_kernel in (L.LONG_STRIPED, L.LONG_PIPELINE) and best.pipe_waves in (0, 2, 4, 8)
    assert L.rawalign_load_tuning(cache).as_dict() == best.as_dict()
    db.score.fill_(-1.0)
    db.run()
    assert _same(db.results(), ref)
