"""GPU parity of the streaming extension (resident rows) and the serving loop."""
import numpy as np
import pytest

from oracle import oracle
from paper_2310_05037_amd import workloads as W

from . import parity
from .serving_oracle import OracleBackend

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


def _extend_round(L, q_chunks, r, r_off, r_len, rows, row_off, first):
    """One rawalign_dtw_extend call; q_chunks[k] is job k's chunk."""
    import torch
    lens = np.array([len(c) for c in q_chunks], np.int32)
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    q = np.concatenate(q_chunks + [np.zeros(1, np.float32)]).astype(np.float32)
    dev = "cuda"
    n = len(q_chunks)
    sc = torch.empty(n, dtype=torch.float32, device=dev)
    en = torch.empty(n, dtype=torch.int32, device=dev)
    L.rawalign_dtw_extend(torch.from_numpy(q).to(dev), torch.from_numpy(offs).to(dev),
                          torch.from_numpy(lens).to(dev), r, torch.from_numpy(r_off).to(dev),
                          torch.from_numpy(r_len).to(dev), rows, torch.from_numpy(row_off).to(dev),
                          torch.from_numpy(first).to(dev), sc, en)
    torch.cuda.synchronize()
    return sc.cpu().numpy(), en.cpu().numpy()


def test_extend_chunked_equals_whole_prefix(L):
    """Streaming a query chunk by chunk through the resident rows gives, after
    every chunk, the float oracle's result on the whole prefix, bit for bit;
    regions span one and several stripes; chunk sizes vary and include
    empty chunks."""
    import torch
    rng = np.random.default_rng(21)
    n_jobs = 24
    ms = rng.integers(1, 9000, n_jobs)
    ms[:6] = [1, 64, 4096, 4097, 8192, 8999]
    r_np = rng.standard_normal(int(ms.sum())).astype(np.float32)
    r_off = np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.int64)
    r_len = ms.astype(np.int32)
    queries = [rng.standard_normal(int(rng.integers(1, 900))).astype(np.float32) for _ in range(n_jobs)]
    row_off = np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.int64) + 5
    rows = torch.full((int(ms.sum()) + 10,), -1.0, device="cuda")
    r = torch.from_numpy(r_np).to("cuda")
    pos = np.zeros(n_jobs, np.int64)
    rounds = 0
    while (pos < [len(x) for x in queries]).any() or rounds == 0:
        sizes = rng.integers(0, 300, n_jobs)
        sizes[rounds % n_jobs] = 0   # an empty chunk somewhere every round
        chunks, first = [], np.zeros(n_jobs, np.uint8)
        for k in range(n_jobs):
            a, b = int(pos[k]), int(min(pos[k] + sizes[k], len(queries[k])))
            chunks.append(queries[k][a:b])
            first[k] = 1 if a == 0 else 0   # no events seen yet: row -1 is zero
            pos[k] = b
        _say(f"  gpu: extend round {rounds} jobs={n_jobs}")
        sc, en = _extend_round(L, chunks, r, r_off, r_len, rows, row_off, first)
        for k in range(n_jobs):
            prefix = queries[k][:int(pos[k])]
            c32, e32 = oracle.dtw_f32(prefix, r_np[r_off[k]:r_off[k] + r_len[k]])
            assert sc[k].view(np.uint32) == np.float32(c32).view(np.uint32) and en[k] == e32, (rounds, k)
        rounds += 1
    # the arena outside the rows is untouched
    assert rows[:5].eq(-1).all() and rows[-5:].eq(-1).all()
    for k in range(n_jobs):
        c64, e64 = oracle.dtw_f64(queries[k], r_np[r_off[k]:r_off[k] + r_len[k]])
        assert abs(float(sc[k]) - c64) <= parity.REL_TOL * c64 + parity.ABS_TOL


def test_extend_alone_equals_mix(L):
    """A job gives the same bits alone and inside a mix of jobs of other
    sizes (continuous batching changes nothing but throughput)."""
    import torch
    rng = np.random.default_rng(22)
    n_jobs = 40
    ms = rng.integers(100, 7000, n_jobs).astype(np.int32)
    r_np = rng.standard_normal(int(ms.sum())).astype(np.float32)
    r_off = np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.int64)
    chunks1 = [rng.standard_normal(int(rng.integers(1, 500))).astype(np.float32) for _ in range(n_jobs)]
    chunks2 = [rng.standard_normal(int(rng.integers(1, 500))).astype(np.float32) for _ in range(n_jobs)]
    r = torch.from_numpy(r_np).to("cuda")
    row_off = r_off.copy()
    rows_mix = torch.zeros(int(ms.sum()), device="cuda")
    _say("  gpu: extend mix")
    _extend_round(L, chunks1, r, r_off, ms, rows_mix, row_off, np.ones(n_jobs, np.uint8))
    mix = _extend_round(L, chunks2, r, r_off, ms, rows_mix, row_off, np.zeros(n_jobs, np.uint8))
    for k in range(0, n_jobs, 7):
        rows1 = torch.zeros(int(ms[k]), device="cuda")
        _say(f"  gpu: extend alone job {k}")
        one = np.array([0], np.int64)
        _extend_round(L, [chunks1[k]], r, r_off[k:k + 1], ms[k:k + 1], rows1, one, np.ones(1, np.uint8))
        a = _extend_round(L, [chunks2[k]], r, r_off[k:k + 1], ms[k:k + 1], rows1, one, np.zeros(1, np.uint8))
        assert a[0][0].view(np.uint32) == mix[0][k].view(np.uint32) and a[1][0] == mix[1][k]
        assert torch.equal(rows1, rows_mix[int(row_off[k]):int(row_off[k]) + int(ms[k])])


def _oracle_engine(wl, b_match=0.4, threshold=20.0):
    from paper_2310_05037_amd import serve

    class VClock:
        t = 0.0

        def __call__(self):
            return self.t
    clock = VClock()
    eng = serve.Engine(OracleBackend(wl.r, 1 << 22), 1 << 22, wl.chunk, wl.period, b_match=b_match,
                       threshold=threshold, clock=clock)
    for i, rd in enumerate(wl.reads):
        eng.submit(i, rd.arrival, rd.events, rd.r_off, rd.r_len)
    while not eng.all_done():
        if eng.tick() == 0:
            clock.t = eng.next_event_time()
    return eng


@pytest.mark.parametrize("use_graph,slots,streams", [(True, 2, 1), (False, 2, 1), (True, 1, 1), (True, 2, 3)])
def test_serving_loop_matches_oracle_engine(L, use_graph, slots, streams):
    """The serving loop on the GPU (real clock, time-compressed arrivals,
    graph-replayed or eager ticks, one or two ticks in flight) returns for
    every read and chunk exactly what the oracle-backed engine returns,
    whatever the tick batching."""
    from paper_2310_05037_amd import serve
    wl = W.serving_workload(60, rate=200.0, chunk=400, max_chunks=4, max_cands=8, ref_bases=200_000,
                            period=1.0, seed_index=33)
    _say(f"  gpu: serving reads={len(wl.reads)} graph={use_graph} slots={slots} streams={streams}")
    eng, st = serve.serve(wl, arena_bytes=64 << 20, time_scale=0.02, use_graph=use_graph, max_jobs=1024,
                          max_reads=128, timeout=120, slots=slots, opts=L.make_opts(streams=streams))
    print("serving", st)
    ref = _oracle_engine(wl)
    assert st["failed"] == 0 and st["ticks"] > 0
    for a, b in zip(eng.reads, ref.reads):
        assert a.status == b.status and len(a.results) == len(b.results), a.rid
        for x, y in zip(a.results, b.results):
            assert x[0] == y[0] and x[1] == y[1] and x[2] == y[2]
            assert np.array_equal(x[3].view(np.uint32), y[3].view(np.uint32)) and np.array_equal(x[4], y[4])


def _same_results(eng, ref):
    for a, b in zip(eng.reads, ref.reads):
        assert a.status == b.status and len(a.results) == len(b.results), a.rid
        for x, y in zip(a.results, b.results):
            assert x[0] == y[0] and x[1] == y[1] and x[2] == y[2]
            assert np.array_equal(x[3].view(np.uint32), y[3].view(np.uint32)) and np.array_equal(x[4], y[4])


def test_serving_streams_chunks_and_binds_memory_cap(L):
    """Reads stream several chunks through the captured ticks: half the
    reads are off target (decoy candidates only, so they never map and run
    to their last chunk) and the match bonus is set for this data's noise
    floor.  Every chunk of every read equals the oracle-backed engine bit
    for bit, with resident rows carried across chunks.  A second run with an
    arena cap of half the first run's peak makes admission wait (reads
    queue), never exceeds the cap, and gives the same results."""
    from paper_2310_05037_amd import serve
    wl = W.serving_workload(48, rate=200.0, chunk=400, max_chunks=5, max_cands=8, ref_bases=200_000,
                            period=1.0, seed_index=34, off_target=0.5)
    bm = W.SYNTHETIC_B_MATCH
    _say(f"  gpu: serving multi-chunk reads={len(wl.reads)} b_match={bm}")
    eng, st = serve.serve(wl, arena_bytes=64 << 20, time_scale=0.02, use_graph=True, max_jobs=1024,
                          max_reads=128, timeout=120, slots=3, opts=L.make_opts(streams=3), b_match=bm)
    print("serving multi-chunk", {k: st[k] for k in ("chunks", "chunks_per_read", "max_chunks_per_read",
                                                      "reads_3plus_chunks", "mapped", "unmapped",
                                                      "peak_arena_bytes", "peak_queued_reads")})
    ref = _oracle_engine(wl, b_match=bm)
    assert st["failed"] == 0 and st["reads_3plus_chunks"] >= 8 and st["unmapped"] >= 10 and st["mapped"] >= 10
    assert all(len(rd.results) > 1 for rd, w in zip(eng.reads, wl.reads) if w.true_cand < 0 and
               len(w.events) > wl.chunk)
    _same_results(eng, ref)
    need = max(int(rd.r_len.sum()) for rd in wl.reads) * 4
    cap = max(st["peak_arena_bytes"] // 2, need)
    assert cap < st["peak_arena_bytes"]
    _say(f"  gpu: serving under a cap of {cap} bytes (uncapped peak {st['peak_arena_bytes']})")
    eng2, st2 = serve.serve(wl, arena_bytes=cap, time_scale=0.02, use_graph=True, max_jobs=1024, max_reads=128,
                            timeout=120, slots=3, opts=L.make_opts(streams=3), b_match=bm)
    print("serving capped", {k: st2[k] for k in ("peak_arena_bytes", "arena_bytes", "peak_queued_reads")})
    assert st2["failed"] == 0 and st2["peak_arena_bytes"] <= cap and st2["peak_queued_reads"] > 0
    _same_results(eng2, ref)


def test_extend_edge_cases(L):
    """A job whose row slot leaves the arena gets the sentinel and writes
    nothing; an empty chunk on a stored row reports that row's minimum and
    leaves it unchanged; an empty chunk with no events seen gives (0, -1);
    an empty region gives (+inf, -1)."""
    import torch
    rng = np.random.default_rng(23)
    ms = np.array([300, 5000, 300, 300, 0], np.int32)
    r_np = rng.standard_normal(int(ms.sum()) + 1).astype(np.float32)
    r_off = np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.int64)
    rows_np = np.abs(rng.standard_normal(6000)).astype(np.float32)
    rows = torch.from_numpy(rows_np.copy()).to("cuda")
    row_off = np.array([5890, 0, 5000, 5400, 10], np.int64)   # job 0's slot ends past the arena
    q = rng.standard_normal(100).astype(np.float32)
    chunks = [q[:50], q[:60], np.zeros(0, np.float32), np.zeros(0, np.float32), q[:10]]
    first = np.array([1, 1, 0, 1, 1], np.uint8)
    sc, en = _extend_round(L, chunks, torch.from_numpy(r_np).to("cuda"), r_off, ms, rows, row_off, first)
    after = rows.cpu().numpy()
    assert np.isnan(sc[0]) and en[0] == -2
    assert np.array_equal(after[5890:], rows_np[5890:])           # job 0 wrote nothing
    from oracle import oracle
    c32, e32 = oracle.dtw_f32(q[:60], r_np[r_off[1]:r_off[1] + ms[1]])
    assert sc[1].view(np.uint32) == np.float32(c32).view(np.uint32) and en[1] == e32
    stored = rows_np[5000:5300]                                     # job 2: empty chunk on a stored row
    assert sc[2] == stored.min() and en[2] == int(np.argmin(stored))
    assert np.array_equal(after[5000:5300], stored)
    assert sc[3] == 0.0 and en[3] == -1                             # nothing seen yet
    assert sc[4] == np.inf and en[4] == -1                          # empty region
