"""CPU model of the pipelined multi-stripe kernel's hand-over protocol
(csrc/dtw_pipe.hip plus the sync hook of the sweep in csrc/dtw_device.h).

Each wave of a workgroup is a generator that performs, in program order,
the kernel's shared-memory operations: the epoch wait and the pair index,
per stripe the progress waits before edge loads, the edge loads and stores
of lanes 0 and 63 row by row, the progress publications every block of steps,
the corner hand-over, the partial minimum, the finished counter, and the
last wave's combine, reset and release of the next pair.  A scheduler runs
the waves in random interleavings (a wave blocked on a wait is not
runnable).  The tests check that every wave terminates with no time-out,
that each edge row a stripe loads was written by its left neighbour for
this pair and not yet overwritten, that every pair's result is written
exactly once after all its waves are done, and that the counters start at
zero for every pair.  No DTW arithmetic is modelled: this is the protocol
only, for the workgroup sizes, block lengths (8 steps in the streaming
extension, 64 in plain batches) and pair shapes the kernel takes.
"""
import random

import pytest

BLOCKS = (8, 64)     # steps between progress publications: streaming extension, plain batches
SKEW = 64            # lane 63 finishes row t - 63 at step t


class Shared:
    def __init__(self, max_stripes=32, waves=4):
        self.epoch = 0
        self.item = None
        self.finished = 0
        self.failed = 0
        self.progress = [0] * max_stripes
        self.corner = {}                       # stripe -> (pair, value tag)
        self.part = [None] * waves


class Model:
    def __init__(self, pairs, W, persistent, grid, rng, block=64):
        self.pairs = pairs                     # list of (n, S)
        self.block = block
        self.W = W
        self.persistent = persistent
        self.grid = grid
        self.rng = rng
        self.queue = 0
        self.edge = {}                         # (workgroup, row) -> (pair, stripe) of the last writer
        self.results = {}                      # pair -> number of writes
        self.active = {}                       # workgroup -> pair being swept

    def next_item(self, wg, item):
        if self.persistent:
            v = self.queue
            self.queue += 1
            return v
        return item + self.grid if item is not None else wg

    def wave(self, wg, w, sh):
        pairs, W = self.pairs, self.W
        n_items = len(pairs)
        seen = 0
        while True:
            while sh.epoch < seen + 1:
                yield "wait"
            seen += 1
            item = sh.item
            if item >= n_items:
                return
            n, S = pairs[item]
            assert self.active.get(wg) in (None, item)
            self.active[wg] = item
            for s in range(w, S, W):
                yield from self.stripe(wg, sh, item, s, n)
            sh.part[w] = (item, w)
            yield "step"
            old = sh.finished
            sh.finished += 1
            yield "step"
            if old == W - 1:
                assert all(sh.part[x] == (item, x) for x in range(W)), "a partial minimum is missing"
                self.results[item] = self.results.get(item, 0) + 1
                del self.active[wg]
                sh.progress = [0] * len(sh.progress)
                sh.finished = 0
                sh.failed = 0
                sh.item = self.next_item(wg, item)
                yield "step"
                sh.epoch = seen + 1

    def wait_progress(self, sh, s, rows):
        while sh.progress[s - 1] < rows:
            yield "wait"

    def stripe(self, wg, sh, pair, s, n):
        # load_lane: the corner for the next stripe is handed over first
        sh.corner[s + 1] = (pair, s)
        if n <= 0:
            return
        if s > 0:
            yield from self.wait_progress(sh, s, min(n, self.block + 2))
            assert sh.corner.get(s) == (pair, s - 1), "corner not handed over"
            # the edges of rows 0 and 1 feed lane 0 at steps 0 and 1 (loads
            # past the last row are clamped and feed masked steps only)
            for row in (0, 1):
                if row < n:
                    self.read(wg, pair, s, row)
        T = (n + SKEW + 1) & ~1
        t = 0
        while t < T:
            if t % self.block == 0:
                if s > 0:
                    yield from self.wait_progress(sh, s, min(n, t + self.block + 2))
                sh.progress[s] = max(0, min(n, t - 63))
            for u in (t, t + 1):
                # lane 0 uses the edge of row u + 2 at step u + 2, for row u + 2
                if s > 0 and u + 2 < n:
                    self.read(wg, pair, s, u + 2)
                row = u - 63
                if 0 <= row < n:
                    self.write(wg, pair, s, row)
            t += 2
            if self.rng.random() < 0.3:
                yield "step"
        sh.progress[s] = n

    def read(self, wg, pair, s, row):
        got = self.edge.get((wg, row))
        assert got == (pair, s - 1), f"stripe {s} of pair {pair} read row {row} written by {got}"

    def write(self, wg, pair, s, row):
        got = self.edge.get((wg, row))
        if s > 0:
            assert got == (pair, s - 1), f"stripe {s} of pair {pair} overwrote row {row} written by {got}"
        self.edge[(wg, row)] = (pair, s)


def run(pairs, W, persistent, grid, seed, block=64):
    rng = random.Random(seed)
    model = Model(pairs, W, persistent, grid, rng, block)
    waves = []
    for wg in range(grid):
        sh = Shared(waves=W)
        # entry: LDS initialised and the first pair released before any wave runs
        sh.item = model.next_item(wg, None)
        sh.epoch = 1
        for w in range(W):
            waves.append((wg, w, model.wave(wg, w, sh)))
    pending = {i: None for i in range(len(waves))}
    stalls = 0
    while pending:
        i = rng.choice(list(pending))
        try:
            ev = next(waves[i][2])
        except StopIteration:
            del pending[i]
            stalls = 0
            continue
        stalls = stalls + 1 if ev == "wait" else 0
        assert stalls < 200000, "no wave can progress: the protocol would hang until the time cap"
    return model


SHAPES = [(1, 3), (2, 2), (63, 5), (64, 4), (65, 3), (100, 9), (200, 1), (130, 2), (257, 12), (1000, 10),
          (0, 4), (513, 32), (70, 7), (3, 16)]


@pytest.mark.parametrize("block", BLOCKS)
@pytest.mark.parametrize("W", [2, 4, 8])
@pytest.mark.parametrize("persistent", [True, False])
def test_pipeline_protocol_random_interleavings(W, persistent, block):
    """Every pair is finished exactly once, every edge load sees its left
    neighbour's value for the same pair, and no wave waits forever, for
    pairs with fewer, as many and more stripes than waves, queries shorter
    than the skew, and one or several workgroups."""
    for seed in range(6):
        grid = 1 + seed % 3
        model = run(SHAPES, W, persistent, grid, seed, block)
        assert model.results == {i: 1 for i in range(len(SHAPES))}


def test_model_catches_a_missing_wait():
    """The model has teeth: a stripe that loads edge rows without waiting
    for its left neighbour is caught on some interleaving."""
    class NoWait(Model):
        def wait_progress(self, sh, s, rows):
            return
            yield
    caught = 0
    for seed in range(10):
        rng = random.Random(seed)
        m = NoWait(SHAPES[:8], 4, True, 1, rng)
        sh = Shared(waves=4)
        sh.item = m.next_item(0, None)
        sh.epoch = 1
        gens = [m.wave(0, w, sh) for w in range(4)]
        alive = list(range(4))
        try:
            while alive:
                i = rng.choice(alive)
                try:
                    next(gens[i])
                except StopIteration:
                    alive.remove(i)
        except AssertionError:
            caught += 1
    assert caught > 0
