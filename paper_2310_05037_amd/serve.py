"""Read Until serving loop: streamed chunks, resident DTW rows, continuous batching.

RawAlign decides per chunk of sequenced signal whether a read maps (Sec. 1:
timely decisions; Sec. 3.1.2: one chunk is the data of about one second of
sequencing; Sec. 2.3: Score = B_Match * N_Read - C_DTW, mapped iff the best
score reaches Score_Threshold).  This module keeps, for every candidate of
every admitted read, the last DTW row of the events seen so far in a device
row arena, so each new chunk extends the alignment instead of redoing it.

Engine (host logic only):
  * admission: a read is admitted when its first chunk is available and the
    arena has room for one row per candidate (4 bytes per region level);
    reads that do not fit wait in arrival order (back-pressure);
  * continuous batching: every tick takes all chunks available at that
    moment from all admitted reads, whatever their sizes, as one job table
    (one job per candidate) and runs the extend and decision kernels once;
  * a read finishes when it maps or after its last chunk; its rows are
    freed and waiting reads may be admitted;
  * per chunk it records the latency from the moment the chunk became
    available to the moment its decision is on the host.
Backends: GpuBackend (librawalign, optionally replaying one captured HIP
graph per tick) and, for tests of the scheduling logic only, a backend
built on the CPU oracle (tests/).
"""
from __future__ import annotations

import bisect
import collections
import gc
import heapq
import time
from dataclasses import dataclass, field

import numpy as np

B_MATCH = 0.4
SCORE_THRESHOLD = 20.0


class ArenaFull(Exception):
    pass


class RowArena:
    """First-fit allocator of float offsets in a buffer of `size` floats."""

    def __init__(self, size: int):
        self.size = int(size)
        self.free = [(0, self.size)]   # sorted (offset, length)
        self.used = 0

    def alloc(self, n: int) -> int:
        n = int(n)
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, ln - n)
                self.used += n
                return off
        raise ArenaFull(n)

    def release(self, off: int, n: int):
        off, n = int(off), int(n)
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, n))
        # merge with neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (off, n + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)
        self.used -= n

    def largest(self) -> int:
        return max((ln for _, ln in self.free), default=0)


@dataclass(eq=False)
class ReadState:
    rid: int
    arrival: float
    events: np.ndarray
    r_off: np.ndarray
    r_len: np.ndarray
    chunk: int
    n_chunks: int = 0
    next_chunk: int = 0          # next chunk index to process
    row_off: np.ndarray | None = None
    admitted: bool = False
    done: bool = False
    status: str = "waiting"      # waiting | active | mapped | unmapped | cancelled | failed
    results: list = field(default_factory=list)   # per chunk: (best_pair, score, mapped, c_dtw[], end[])
    inflight: bool = False       # a launched tick holds this read's chunk (its kernels may write its rows)
    release_pending: bool = False   # finished while in flight: free the rows when that tick returns

    def chunk_ready_time(self, c: int, period: float) -> float:
        return self.arrival + c * period


@dataclass
class TickBatch:
    """Jobs of one tick.  Read t of the tick owns jobs cand_off[t] ..
    cand_off[t]+cand_cnt[t]-1; its chunk events are chunks[t]."""
    reads: list
    chunks: list
    r_off: np.ndarray
    r_len: np.ndarray
    row_off: np.ndarray
    first: np.ndarray
    cand_off: np.ndarray
    cand_cnt: np.ndarray
    n_events: np.ndarray

    @property
    def n_jobs(self) -> int:
        return int(len(self.r_off))

    @property
    def cells(self) -> int:
        lens = np.repeat(np.array([len(c) for c in self.chunks], np.int64), self.cand_cnt)
        return int(np.dot(lens, self.r_len.astype(np.int64)))


class Engine:
    def __init__(self, backend, arena_floats: int, chunk: int = 400, period: float = 1.0,
                 b_match: float = B_MATCH, threshold: float = SCORE_THRESHOLD, max_jobs: int = 1 << 15,
                 max_reads: int = 4096, clock=None):
        self.backend = backend
        self.arena = RowArena(arena_floats)
        self.chunk = chunk
        self.period = period
        self.b_match = b_match
        self.threshold = threshold
        self.max_jobs = max_jobs
        self.max_reads = max_reads
        self.clock = clock or time.perf_counter
        self.reads: list[ReadState] = []     # in submission order
        self.by_id: dict[int, ReadState] = {}
        self.future: list[ReadState] = []    # not yet available, sorted by arrival
        self.next_future = 0
        self.pending = collections.deque()   # available, waiting for arena room (arrival order)
        self.heap = []                       # (next chunk ready time, seq, read id) of admitted reads
        self.seq = 0
        self.n_done = 0
        self.latencies = []                  # (read id, chunk, latency seconds)
        self.ticks = 0
        self.cells = 0
        self.jobs = 0
        self.rejected = 0
        self.peak_arena = 0
        self.peak_pending = 0                # most reads waiting for arena room at once
        self.failed_ticks = 0
        # Backends with launch/poll run up to `slots` ticks at once.
        self.async_backend = hasattr(backend, "launch") and getattr(backend, "slots", 1) > 1
        self.slots = getattr(backend, "slots", 1) if self.async_backend else 1
        self.inflight = collections.deque()   # (token, TickBatch) launched, results pending

    # ---- submission ------------------------------------------------------------
    def submit(self, rid: int, arrival: float, events: np.ndarray, r_off, r_len):
        """Register a read whose first chunk is available at `arrival`; chunk
        c is available at arrival + c * period.  Submit in arrival order."""
        r_off = np.asarray(r_off, np.int64)
        r_len = np.asarray(r_len, np.int32)
        st = ReadState(rid, arrival, np.ascontiguousarray(events, np.float32), r_off, r_len, self.chunk)
        st.n_chunks = (len(events) + self.chunk - 1) // self.chunk
        self.reads.append(st)
        self.by_id[rid] = st
        if int(r_len.sum()) > self.arena.size or st.n_chunks == 0:
            st.status = "failed"     # can never fit (or nothing to do): refuse instead of blocking the queue
            st.done = True
            self.n_done += 1
            self.rejected += 1
        else:
            if self.future and arrival < self.future[-1].arrival:
                raise ValueError("submit reads in arrival order")
            self.future.append(st)
        return st

    def cancel(self, rid: int):
        """Stop a read.  If a tick holding its chunk is still running, its
        rows stay allocated until that tick returns, since the running
        kernels still write them."""
        st = self.by_id.get(rid)
        if st is not None and not st.done:
            self._finish(st, "cancelled")

    # ---- scheduling ------------------------------------------------------------
    def _release(self, st: ReadState):
        if st.admitted and st.row_off is not None:
            # one block per read: the candidates' rows are contiguous
            self.arena.release(int(st.row_off[0]), int(st.r_len.astype(np.int64).sum()))
        st.row_off = None
        st.release_pending = False

    def _returned(self, b: "TickBatch"):
        """The tick of batch b is over: its reads' rows are no longer written."""
        for st in b.reads:
            st.inflight = False
            if st.release_pending:
                self._release(st)

    def _finish(self, st: ReadState, status: str):
        if st.inflight:
            st.release_pending = True   # freed by _returned when its tick is back
        else:
            self._release(st)
        st.done = True
        st.status = status
        self.n_done += 1
        if not st.admitted and st in self.pending:
            self.pending.remove(st)

    def _push(self, st: ReadState):
        heapq.heappush(self.heap, (st.chunk_ready_time(st.next_chunk, self.period), self.seq, st.rid))
        self.seq += 1

    def _admit(self, now: float):
        while self.next_future < len(self.future) and self.future[self.next_future].arrival <= now:
            st = self.future[self.next_future]
            self.next_future += 1
            if not st.done:
                self.pending.append(st)
        self.peak_pending = max(self.peak_pending, len(self.pending))
        # arrival order: nobody overtakes a read that does not fit yet
        while self.pending:
            st = self.pending[0]
            lens = st.r_len.astype(np.int64)
            try:
                base = self.arena.alloc(int(lens.sum()))   # one block for all the read's rows
            except ArenaFull:
                break
            self.pending.popleft()
            st.row_off = base + np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
            st.admitted = True
            st.status = "active"
            self._push(st)
        self.peak_arena = max(self.peak_arena, self.arena.used)

    def _ready(self, now: float):
        out, jobs = [], 0
        while self.heap and self.heap[0][0] <= now and len(out) < self.max_reads:
            _, _, rid = self.heap[0]
            st = self.by_id[rid]
            if st.done:
                heapq.heappop(self.heap)
                continue
            if out and jobs + len(st.r_len) > self.max_jobs:
                break
            heapq.heappop(self.heap)
            out.append(st)
            jobs += len(st.r_len)
        return out

    def _batch(self, ready) -> TickBatch:
        chunks, first, cand_cnt, n_ev = [], [], [], []
        for st in ready:
            c = st.next_chunk
            chunks.append(st.events[c * self.chunk:(c + 1) * self.chunk])
            first.append(np.full(len(st.r_len), 1 if c == 0 else 0, np.uint8))
            cand_cnt.append(len(st.r_len))
            n_ev.append(min((c + 1) * self.chunk, len(st.events)))
        cc = np.array(cand_cnt, np.int32)
        return TickBatch(list(ready), chunks, np.concatenate([st.r_off for st in ready]),
                         np.concatenate([st.r_len for st in ready]), np.concatenate([st.row_off for st in ready]),
                         np.concatenate(first), np.concatenate([[0], np.cumsum(cc)[:-1]]).astype(np.int64), cc,
                         np.array(n_ev, np.int32))

    def _fail(self, b: TickBatch):
        """A backend error fails only the reads of that tick."""
        self.failed_ticks += 1
        self._returned(b)
        for st in b.reads:
            if not st.done:
                self._finish(st, "failed")

    def _complete(self, b: TickBatch, results, t_done: float) -> int:
        score, end, best, best_score, mapped = results
        self._returned(b)
        self.ticks += 1
        self.jobs += b.n_jobs
        self.cells += b.cells
        for t, st in enumerate(b.reads):
            lo, k = int(b.cand_off[t]), int(b.cand_cnt[t])
            c = st.next_chunk
            st.results.append((int(best[t]) - lo if best[t] >= 0 else -1, float(best_score[t]), int(mapped[t]),
                               score[lo:lo + k].copy(), end[lo:lo + k].copy()))
            self.latencies.append((st.rid, c, t_done - st.chunk_ready_time(c, self.period)))
            st.next_chunk += 1
            if st.done:                      # cancelled while its chunk was in flight
                continue
            if mapped[t]:
                self._finish(st, "mapped")
            elif st.next_chunk >= st.n_chunks:
                self._finish(st, "unmapped")
            else:
                self._push(st)
        return len(b.reads)

    def tick(self) -> int:
        """One scheduling step: collect the ticks that finished, then start
        one with every chunk available now (if a slot is free).  Returns the
        number of chunks completed or started."""
        done = 0
        if self.inflight:
            still = collections.deque()
            for token, b in self.inflight:
                try:
                    res = self.backend.poll(token)
                except Exception:
                    self._fail(b)
                    continue
                if res is None:
                    still.append((token, b))
                else:
                    done += self._complete(b, res, self.clock())
            self.inflight = still
        now = self.clock()
        self._admit(now)
        if len(self.inflight) >= self.slots:
            return done
        ready = self._ready(now)
        if not ready:
            return done
        b = self._batch(ready)
        for st in b.reads:
            st.inflight = True
        if self.async_backend:
            try:
                token = self.backend.launch(b, self.b_match, self.threshold)
            except Exception:
                self._fail(b)
                return done
            self.inflight.append((token, b))
            return done + len(b.reads)
        try:
            res = self.backend.run(b, self.b_match, self.threshold)
        except Exception:
            self._fail(b)
            return done
        return done + self._complete(b, res, self.clock())

    def all_done(self) -> bool:
        return self.n_done == len(self.reads)

    def next_event_time(self) -> float | None:
        t = []
        if self.heap:
            t.append(self.heap[0][0])
        if self.next_future < len(self.future):
            t.append(self.future[self.next_future].arrival)
        return min(t) if t else None

    def run(self, idle_sleep: float = 2e-4, poll_sleep: float = 0.0, timeout: float | None = None,
            spin: float = 1.5e-4):
        """Serve until every read is done.  While ticks are in flight the
        loop polls them without sleeping (poll_sleep 0).  While it waits for
        the next chunk it sleeps until `spin` seconds before that chunk and
        polls the clock from there: a sleep overruns by tens of microseconds
        (timer slack), and every overrun is added to a chunk's latency.  The
        loop therefore keeps one host core busy while reads are in flight."""
        t0 = self.clock()
        while not self.all_done() or self.inflight:
            if self.tick() == 0:
                if timeout is not None and self.clock() - t0 > timeout:
                    raise TimeoutError("serving loop did not finish")
                if self.inflight:
                    if poll_sleep > 0:
                        time.sleep(poll_sleep)
                    continue
                nxt = self.next_event_time()
                if nxt is None and self.pending:
                    raise RuntimeError("reads wait for arena room that no running read will free")
                wait = idle_sleep if nxt is None else min(max(nxt - self.clock(), 0.0), idle_sleep)
                if wait > spin:
                    time.sleep(wait - spin)

    def stats(self) -> dict:
        lat = np.array([x[2] for x in self.latencies]) if self.latencies else np.zeros(1)
        st = [s.status for s in self.reads]
        per_read = np.array([len(s.results) for s in self.reads]) if self.reads else np.zeros(1)
        return {"chunks": len(self.latencies), "reads": len(self.reads), "ticks": self.ticks, "jobs": self.jobs,
                "chunks_per_read": float(per_read.mean()), "max_chunks_per_read": int(per_read.max()),
                "reads_3plus_chunks": int((per_read >= 3).sum()), "peak_queued_reads": int(self.peak_pending),
                "cells": self.cells, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "p999_ms": float(np.percentile(lat, 99.9) * 1e3),
                "max_ms": float(lat.max() * 1e3), "mapped": st.count("mapped"), "unmapped": st.count("unmapped"),
                "failed": st.count("failed"), "cancelled": st.count("cancelled"),
                "peak_arena_bytes": int(self.peak_arena) * 4, "arena_bytes": self.arena.size * 4}


class _Slot:
    """Tables, outputs, stream and graph of one tick in flight.  The input
    tables live in one pinned host buffer and one device buffer of the same
    layout (one copy per direction per tick), likewise the outputs."""

    IN = (("q", "float32", "R*chunk"), ("q_off", "int64", "J"), ("r_off", "int64", "J"), ("row_off", "int64", "J"),
          ("cand_off", "int64", "R"), ("q_len", "int32", "J"), ("r_len", "int32", "J"), ("cand_cnt", "int32", "R"),
          ("n_events", "int32", "R"), ("first", "uint8", "J"))
    OUT = (("best_score", "float64", "R"), ("score", "float32", "J"), ("end", "int32", "J"), ("best", "int32", "R"),
           ("mapped", "uint8", "R"))

    @staticmethod
    def _views(torch, fields, sizes, device, pin):
        """One byte buffer split into 256-byte aligned typed views."""
        spans, off = [], 0
        for name, dt, n in fields:
            dtype = getattr(torch, dt)
            count = sizes[n]
            nbytes = count * torch.empty(0, dtype=dtype).element_size()
            spans.append((name, dtype, off, nbytes))
            off += (nbytes + 255) // 256 * 256
        buf = torch.empty(off, dtype=torch.uint8, device=device, pin_memory=pin)
        return buf, {name: buf[o:o + nb].view(dtype) for name, dtype, o, nb in spans}

    def __init__(self, torch, dev, chunk, J, R):
        sizes = {"R*chunk": R * chunk, "J": J, "R": R}
        self.h_buf, self.h = self._views(torch, self.IN, sizes, "cpu", True)
        self.d_buf, self.d = self._views(torch, self.IN, sizes, dev, False)
        self.do_buf, self.d_out = self._views(torch, self.OUT, sizes, dev, False)
        self.ho_buf, self.h_out = self._views(torch, self.OUT, sizes, "cpu", True)
        self.h_buf.zero_()
        self.stream = torch.cuda.Stream()
        self.start = torch.cuda.Event(enable_timing=True)
        self.event = torch.cuda.Event(enable_timing=True)
        self.graph = None
        self.busy = False
        self.shape = (0, 0)   # jobs and reads of the tick in flight


class GpuBackend:
    """librawalign on one device: rawalign_dtw_extend over the tick's jobs,
    then rawalign_decide over its reads.  With use_graph, a tick (pinned
    host-to-device copies, both library calls, device-to-host copies) is
    captured once into a HIP graph over fixed-capacity tables and replayed;
    unused job slots carry q_len = -1 (sentinel, no kernel work) and unused
    read slots no candidates.  With slots > 1, up to that many ticks are in
    flight at once, each with its own tables, stream and graph (launch/poll):
    a chunk that becomes available while a tick runs does not wait for it.
    Ticks in flight never share a read (a read's next chunk is scheduled only
    after its results are back), so their rows are disjoint."""

    def __init__(self, r_levels: np.ndarray, arena_floats: int, chunk: int = 400, max_jobs: int = 1 << 15,
                 max_reads: int = 4096, use_graph: bool = True, opts=None, slots: int = 2):
        import torch
        from . import lib
        self.torch, self.lib = torch, lib
        dev = torch.device("cuda", torch.cuda.current_device())
        self.chunk, self.max_jobs, self.max_reads = chunk, max_jobs, max_reads
        self.r = torch.from_numpy(np.ascontiguousarray(r_levels, np.float32)).to(dev)
        self.rows = torch.zeros(int(arena_floats), dtype=torch.float32, device=dev)
        self.opts = opts
        self.use_graph = use_graph
        self.slots = int(slots)
        self.slot = [_Slot(torch, dev, chunk, max_jobs, max_reads) for _ in range(self.slots)]
        self.params = None
        self.tick_ms = []   # device time of every tick (first copy to last copy)

    def _work(self, sl: _Slot, b_match, threshold):
        d, o = sl.d, sl.d_out
        sl.d_buf.copy_(sl.h_buf, non_blocking=True)
        self.lib.rawalign_dtw_extend(d["q"], d["q_off"], d["q_len"], self.r, d["r_off"], d["r_len"], self.rows,
                                     d["row_off"], d["first"], o["score"], o["end"], opts=self.opts)
        self.lib.rawalign_decide(o["score"], d["cand_off"], d["cand_cnt"], d["n_events"], o["best"],
                                 o["best_score"], o["mapped"], b_match=b_match, threshold=threshold)
        sl.ho_buf.copy_(sl.do_buf, non_blocking=True)

    def _fill(self, sl: _Slot, b: TickBatch):
        h = sl.h
        nj, nr = b.n_jobs, len(b.reads)
        if nj > self.max_jobs or nr > self.max_reads:
            raise ValueError("tick larger than the backend tables")
        q = h["q"].numpy()
        lens = np.zeros(nr, np.int32)
        for t, ev in enumerate(b.chunks):
            q[t * self.chunk:t * self.chunk + len(ev)] = ev
            lens[t] = len(ev)
        job_read = np.repeat(np.arange(nr), b.cand_cnt)
        h["q_off"].numpy()[:nj] = job_read * self.chunk
        ql = h["q_len"].numpy()
        ql[:nj] = lens[job_read]
        ql[nj:] = -1                           # empty slots: sentinel, no kernel work
        h["r_off"].numpy()[:nj] = b.r_off
        h["r_len"].numpy()[:nj] = b.r_len
        h["row_off"].numpy()[:nj] = b.row_off
        h["first"].numpy()[:nj] = b.first
        h["cand_off"].numpy()[:nr] = b.cand_off
        cc = h["cand_cnt"].numpy()
        cc[:nr] = b.cand_cnt
        cc[nr:] = 0
        h["n_events"].numpy()[:nr] = b.n_events

    def prepare(self, b_match: float, threshold: float):
        """Per slot: warm up over blank tables (every slot a sentinel, the
        rows untouched) so the library allocates its scratch outside any
        capture, then capture one tick into a graph and replay it once (the
        first replay uploads it).  The graph reads the pinned host tables
        when it is replayed, so it serves every later tick of that slot."""
        torch = self.torch
        for sl in self.slot:
            sl.h["q_len"].fill_(-1)
            sl.h["cand_cnt"].fill_(0)
            with torch.cuda.stream(sl.stream):
                self._work(sl, b_match, threshold)
                sl.stream.synchronize()
                if self.use_graph:
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=sl.stream):
                        self._work(sl, b_match, threshold)
                    sl.graph = g
                    g.replay()
                    sl.stream.synchronize()
        self.params = (b_match, threshold)

    def launch(self, b: TickBatch, b_match: float, threshold: float) -> int:
        if self.params != (b_match, threshold):
            if any(sl.busy for sl in self.slot):
                raise RuntimeError("decision parameters changed while ticks are in flight")
            self.prepare(b_match, threshold)
        i = next((k for k, sl in enumerate(self.slot) if not sl.busy), None)
        if i is None:
            raise RuntimeError("no free tick slot")
        sl = self.slot[i]
        self._fill(sl, b)
        with self.torch.cuda.stream(sl.stream):
            sl.start.record(sl.stream)
            if self.use_graph:
                sl.graph.replay()
            else:
                self._work(sl, b_match, threshold)
            sl.event.record(sl.stream)
        sl.busy = True
        sl.shape = (b.n_jobs, len(b.reads))
        return i

    def poll(self, i: int):
        """Results of the tick in slot i, or None while it runs."""
        sl = self.slot[i]
        if not sl.event.query():
            return None
        sl.busy = False
        self.tick_ms.append(sl.start.elapsed_time(sl.event))
        nj, nr = sl.shape
        o = sl.h_out
        return (o["score"].numpy()[:nj].copy(), o["end"].numpy()[:nj].copy(), o["best"].numpy()[:nr].copy(),
                o["best_score"].numpy()[:nr].copy(), o["mapped"].numpy()[:nr].copy())

    def run(self, b: TickBatch, b_match: float, threshold: float):
        """Synchronous tick (one slot at a time)."""
        i = self.launch(b, b_match, threshold)
        self.slot[i].event.synchronize()
        return self.poll(i)


def serve(workload, arena_bytes: int = 8 << 30, time_scale: float = 1.0, use_graph: bool = True,
          max_jobs: int = 8192, max_reads: int = 256, timeout: float | None = None, backend=None,
          slots: int = 3, opts=None, b_match: float = B_MATCH, threshold: float = SCORE_THRESHOLD):
    """Run a workloads.ServingWorkload through the engine on the GPU.
    time_scale compresses the arrival and chunk clock (0.01: a 1 s chunk
    period becomes 10 ms); slots is the number of ticks in flight; opts
    (lib.Opts) goes to the extension call; b_match and threshold are the
    decision's match bonus and score threshold (Sec. 2.3).
    max_jobs/max_reads size the per-tick tables (a captured tick copies them
    whole); chunks beyond them wait for the next tick."""
    arena_floats = arena_bytes // 4
    if backend is None:
        backend = GpuBackend(workload.r, arena_floats, workload.chunk, max_jobs, max_reads, use_graph, opts=opts,
                             slots=slots)
    # The engine's clock starts at zero when the loop starts, after every read
    # has been submitted (submitting many reads takes a while itself).
    origin = [time.perf_counter()]

    def clock():
        return time.perf_counter() - origin[0]

    eng = Engine(backend, arena_floats, workload.chunk, workload.period * time_scale, b_match=b_match,
                 threshold=threshold, max_jobs=max_jobs, max_reads=max_reads, clock=clock)
    if hasattr(backend, "prepare"):
        backend.prepare(eng.b_match, eng.threshold)   # capture before the clock starts
    for i, rd in enumerate(workload.reads):
        eng.submit(i, rd.arrival * time_scale, rd.events, rd.r_off, rd.r_len)
    # No garbage-collection pauses inside the timed loop: a full collection
    # over the run's many small arrays can stall the host for tens of ms.
    gc.collect()
    gc.disable()
    try:
        origin[0] = time.perf_counter()
        eng.run(timeout=timeout)
        wall = eng.clock()
    finally:
        gc.enable()
    st = eng.stats()
    # The five slowest chunks: (moment the chunk became available, relative
    # to the start of the run, and its latency), in ms.
    worst = sorted(eng.latencies, key=lambda x: -x[2])[:5]
    st["worst_ms"] = [(round(eng.reads[rid].chunk_ready_time(c, eng.period) * 1e3, 3), round(lat * 1e3, 3))
                      for rid, c, lat in worst]
    st.update({"wall_s": wall, "gcups": eng.cells / wall / 1e9, "chunks_per_s": st["chunks"] / wall,
               "time_scale": time_scale, "rate_reads_per_s": workload.rate / time_scale})
    tick_ms = getattr(backend, "tick_ms", None)
    if tick_ms:
        st["tick_device_ms"] = {"p50": float(np.percentile(tick_ms, 50)), "p99": float(np.percentile(tick_ms, 99)),
                                "max": float(np.max(tick_ms))}
    return eng, st
