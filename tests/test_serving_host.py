"""Host logic of the Read Until serving loop, run against the CPU oracle
backend with a virtual clock (no GPU)."""
import numpy as np
import pytest

from oracle import oracle
from paper_2310_05037_amd import serve
from paper_2310_05037_amd import workloads as W

from .serving_oracle import OracleBackend


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def drive(eng, clock, dt=None, max_ticks=100000):
    """Advance the virtual clock to the next event (or by dt) and tick."""
    for _ in range(max_ticks):
        if eng.all_done() and not eng.inflight:
            return
        if eng.tick() == 0:
            if eng.inflight:          # waiting for launched ticks: keep polling
                if dt:
                    clock.t += dt
                continue
            if eng.all_done():        # the last tick failed: nothing left to run
                continue
            nxt = eng.next_event_time()
            if nxt is None:
                raise RuntimeError("stuck")
            clock.t = clock.t + dt if dt else nxt
    raise RuntimeError("too many ticks")


def small_workload(n_reads=12, seed_index=3):
    return W.serving_workload(n_reads, rate=50.0, chunk=40, max_chunks=4, max_cands=5, ref_bases=20_000,
                              period=0.1, seed_index=seed_index)


def test_row_arena_first_fit_and_merge():
    a = serve.RowArena(100)
    o1 = a.alloc(30)
    o2 = a.alloc(30)
    o3 = a.alloc(40)
    assert (o1, o2, o3) == (0, 30, 60) and a.used == 100
    with pytest.raises(serve.ArenaFull):
        a.alloc(1)
    a.release(o2, 30)
    assert a.alloc(20) == 30 and a.largest() == 10
    a.release(o1, 30)
    a.release(30, 20)
    a.release(o3, 40)
    assert a.free == [(0, 100)] and a.used == 0


def test_results_equal_whole_prefix_oracle():
    """Every chunk's cost and end equal the float oracle on the whole prefix
    seen so far (streaming == whole), and the decision follows Sec. 2.3."""
    wl = small_workload()
    clock = VClock()
    be = OracleBackend(wl.r, 1 << 20)
    eng = serve.Engine(be, 1 << 20, wl.chunk, wl.period, clock=clock)
    for i, rd in enumerate(wl.reads):
        eng.submit(i, rd.arrival, rd.events, rd.r_off, rd.r_len)
    drive(eng, clock, dt=wl.period / 2)   # coarse ticks: chunks of several reads wait together
    assert max(be.batch_sizes) > 1   # several reads shared a tick
    for st in eng.reads:
        assert st.status in ("mapped", "unmapped")
        for c, (best, bscore, mapped, cost, end) in enumerate(st.results):
            n = min((c + 1) * wl.chunk, len(st.events))
            prefix = st.events[:n]
            exp = [oracle.dtw_f32(prefix, wl.r[o:o + l]) for o, l in zip(st.r_off, st.r_len)]
            assert np.array_equal(cost, np.array([x[0] for x in exp], np.float32))
            assert np.array_equal(end, np.array([x[1] for x in exp], np.int32))
            b, s, m = oracle.decide(cost, [0], [len(cost)], [n])
            assert best == b[0] and bscore == s[0] and mapped == m[0]
        if st.status == "mapped":
            assert st.results[-1][2] == 1
        else:
            assert len(st.results) == st.n_chunks and all(r[2] == 0 for r in st.results)


def test_admission_respects_memory_cap_and_order():
    """With an arena that holds about one read, reads run one after another,
    the arena never overflows, and nobody overtakes the head of the queue."""
    wl = small_workload(n_reads=8)
    need = max(int(rd.r_len.sum()) for rd in wl.reads)
    clock = VClock()
    be = OracleBackend(wl.r, need)
    eng = serve.Engine(be, need, wl.chunk, wl.period, clock=clock)
    for i, rd in enumerate(wl.reads):
        eng.submit(i, rd.arrival, rd.events, rd.r_off, rd.r_len)
    admitted_order = []
    for _ in range(100000):
        if eng.all_done():
            break
        before = {st.rid for st in eng.reads if st.admitted}
        n = eng.tick()
        assert eng.arena.used <= need
        admitted_order += sorted({st.rid for st in eng.reads if st.admitted} - before)
        if n == 0:
            clock.t = eng.next_event_time() if eng.next_event_time() is not None else clock.t + wl.period
    assert eng.all_done()
    assert admitted_order == sorted(admitted_order)
    assert eng.stats()["peak_arena_bytes"] <= need * 4


def test_read_that_cannot_fit_is_refused_not_blocking():
    wl = small_workload(n_reads=4)
    cap = int(max(int(rd.r_len.sum()) for rd in wl.reads[1:]))
    big = wl.reads[0]
    clock = VClock()
    eng = serve.Engine(OracleBackend(wl.r, cap), cap, wl.chunk, wl.period, clock=clock)
    eng.submit(0, big.arrival, big.events, big.r_off, np.full_like(big.r_len, cap))  # larger than the arena
    for i, rd in enumerate(wl.reads[1:], 1):
        eng.submit(i, rd.arrival, rd.events, rd.r_off, rd.r_len)
    drive(eng, clock)
    assert eng.reads[0].status == "failed" and eng.rejected == 1
    assert all(st.status in ("mapped", "unmapped") for st in eng.reads[1:])


def test_cancel_frees_rows():
    wl = small_workload(n_reads=3)
    clock = VClock()
    eng = serve.Engine(OracleBackend(wl.r, 1 << 20), 1 << 20, wl.chunk, wl.period, clock=clock)
    for i, rd in enumerate(wl.reads):
        eng.submit(i, 0.0, rd.events, rd.r_off, rd.r_len)
    eng.tick()
    assert eng.arena.used > 0
    for st in eng.reads:
        eng.cancel(st.rid)
    assert eng.arena.used == 0 and all(st.status in ("cancelled", "mapped", "unmapped") for st in eng.reads)
    assert eng.all_done()


def test_backend_failure_fails_only_that_tick():
    wl = small_workload(n_reads=10)
    clock = VClock()
    be = OracleBackend(wl.r, 1 << 20, fail_on_call=2)
    eng = serve.Engine(be, 1 << 20, wl.chunk, wl.period, clock=clock)
    for i, rd in enumerate(wl.reads):
        eng.submit(i, rd.arrival, rd.events, rd.r_off, rd.r_len)
    drive(eng, clock)
    st = eng.stats()
    assert eng.failed_ticks == 1 and st["failed"] >= 1
    assert st["failed"] + st["mapped"] + st["unmapped"] == len(wl.reads)
    assert eng.arena.used == 0


def test_latency_accounting_virtual_clock():
    """A chunk processed at the moment it becomes available has zero latency."""
    wl = small_workload(n_reads=5)
    clock = VClock()
    eng = serve.Engine(OracleBackend(wl.r, 1 << 20), 1 << 20, wl.chunk, wl.period, clock=clock)
    for i, rd in enumerate(wl.reads):
        eng.submit(i, rd.arrival, rd.events, rd.r_off, rd.r_len)
    drive(eng, clock)
    assert all(abs(x[2]) < 1e-12 for x in eng.latencies)
    assert eng.stats()["chunks"] == sum(len(st.results) for st in eng.reads)


def test_chain_order_keeps_reads_and_places_true_region():
    """The synthetic chaining order permutes candidates only within their
    read, keeps every pair, and puts the true region first for about the
    requested share of reads."""
    b = W.plain_batch(n_pairs=2000)
    c = W.chain_ordered(b, seed=3, p_true_first=0.8)
    assert np.array_equal(c.cand_off, b.cand_off) and np.array_equal(c.cand_cnt, b.cand_cnt)
    for k in range(len(b.cand_off)):
        p0, n = int(b.cand_off[k]), int(b.cand_cnt[k])
        got = sorted(zip(c.r_off[p0:p0 + n].tolist(), c.q_off[p0:p0 + n].tolist(), c.r_len[p0:p0 + n].tolist()))
        exp = sorted(zip(b.r_off[p0:p0 + n].tolist(), b.q_off[p0:p0 + n].tolist(), b.r_len[p0:p0 + n].tolist()))
        assert got == exp
        t = int(c.true_pair[k])
        assert p0 <= t < p0 + n and c.r_off[t] == b.r_off[b.true_pair[k]]
    share = float((c.true_pair == c.cand_off).mean())
    assert 0.65 < share < 0.95


class AsyncOracle(OracleBackend):
    """Oracle backend with launch/poll: a tick's results appear only after a
    few polls, so several ticks are in flight at once."""
    slots = 2

    def __init__(self, *a, delay=3, **k):
        super().__init__(*a, **k)
        self.delay = delay
        self.pending = {}
        self.next_token = 0
        self.max_inflight = 0

    def launch(self, b, b_match, threshold):
        res = self.run(b, b_match, threshold)
        tok = self.next_token
        self.next_token += 1
        self.pending[tok] = [self.delay, res]
        self.max_inflight = max(self.max_inflight, len(self.pending))
        return tok

    def poll(self, tok):
        entry = self.pending[tok]
        if entry[0] > 0:
            entry[0] -= 1
            return None
        del self.pending[tok]
        return entry[1]


def test_ticks_in_flight_give_the_same_results():
    """With two ticks in flight (launch/poll) every read gets the same
    per-chunk results and status as with synchronous ticks, and no more than
    two ticks are ever in flight."""
    wl = small_workload(n_reads=16, seed_index=5)
    runs = []
    for be in (OracleBackend(wl.r, 1 << 20), AsyncOracle(wl.r, 1 << 20)):
        clock = VClock()
        eng = serve.Engine(be, 1 << 20, wl.chunk, wl.period, clock=clock)
        assert eng.slots == (2 if isinstance(be, AsyncOracle) else 1)
        for i, rd in enumerate(wl.reads):
            eng.submit(i, rd.arrival, rd.events, rd.r_off, rd.r_len)
        drive(eng, clock, dt=wl.period / 7)
        assert not eng.inflight
        runs.append((eng, be))
    (e1, _), (e2, be2) = runs
    assert be2.max_inflight == 2
    for a, b in zip(e1.reads, e2.reads):
        assert a.status == b.status and len(a.results) == len(b.results)
        for x, y in zip(a.results, b.results):
            assert x[:3] == y[:3] and np.array_equal(x[3], y[3]) and np.array_equal(x[4], y[4])


class OverlapCheckingAsync(AsyncOracle):
    """Async oracle backend that asserts, at every launch, that the new
    tick's rows are disjoint from the rows of every tick still in flight
    (on a GPU those kernels would still be writing them)."""
    slots = 3

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.live = {}

    def launch(self, b, b_match, threshold):
        iv = [(int(o), int(o) + int(n)) for o, n in zip(b.row_off, b.r_len)]
        for other in self.live.values():
            for a0, a1 in iv:
                for b0, b1 in other:
                    assert a1 <= b0 or b1 <= a0, "rows of a new tick overlap a tick in flight"
        tok = super().launch(b, b_match, threshold)
        self.live[tok] = iv
        return tok

    def poll(self, tok):
        res = super().poll(tok)
        if res is not None:
            del self.live[tok]
        return res


def test_cancel_in_flight_keeps_rows_until_the_tick_returns():
    """A read cancelled while its tick runs keeps its rows until that tick
    returns: a waiting read that would fit in the freed block is admitted
    only afterwards, so no two ticks in flight ever share rows."""
    wl = small_workload(n_reads=3)
    need = sum(int(rd.r_len.sum()) for rd in wl.reads)
    clock = VClock()
    be = OverlapCheckingAsync(wl.r, need, delay=5)
    eng = serve.Engine(be, need, wl.chunk, wl.period, clock=clock)
    for i, rd in enumerate(wl.reads):
        eng.submit(i, 0.0, rd.events, rd.r_off, rd.r_len)
    r0 = wl.reads[0]
    eng.submit(3, 0.0, r0.events, r0.r_off, r0.r_len)   # fits exactly in read 0's block
    eng.tick()
    assert all(st.inflight for st in eng.reads[:3]) and eng.arena.used == need
    eng.cancel(0)
    assert eng.reads[0].status == "cancelled" and eng.reads[0].release_pending
    assert eng.arena.used == need                        # still written by the running tick
    eng.tick()
    assert not eng.reads[3].admitted
    drive(eng, clock)
    assert eng.reads[0].status == "cancelled" and eng.reads[3].admitted
    assert eng.reads[3].status in ("mapped", "unmapped")
    assert eng.arena.used == 0 and not be.live


def test_failed_tick_releases_cancelled_rows():
    """A tick that fails returns its reads' rows too, cancelled ones included."""
    wl = small_workload(n_reads=3)
    clock = VClock()

    class FailingAsync(OverlapCheckingAsync):
        def poll(self, tok):
            res = super().poll(tok)
            if res is not None:
                raise RuntimeError("injected failure")
            return res

    be = FailingAsync(wl.r, 1 << 20, delay=2)
    eng = serve.Engine(be, 1 << 20, wl.chunk, wl.period, clock=clock)
    for i, rd in enumerate(wl.reads):
        eng.submit(i, 0.0, rd.events, rd.r_off, rd.r_len)
    eng.tick()
    eng.cancel(1)
    assert eng.arena.used > 0
    drive(eng, clock)
    assert eng.arena.used == 0 and eng.failed_ticks >= 1
    assert eng.reads[1].status == "cancelled"
