"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Each test names the mathematical fact it relies on.  Together they are meant
to catch a plausible mistake anywhere in the recurrence: a dropped neighbour,
a wrong boundary value, a swapped operand, a wrong tie rule or an off-by-one
in the rolling rows.
"""
import math
import os

import numpy as np
import pytest

from oracle import brute
from paper_2310_05037_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.txt")


def _golden_cases():
    cases, cur = [], None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            if cur:
                cases.append(cur)
                cur = None
            continue
        key, *vals = line.split()
        if key == "case":
            cur = {"name": vals[0], "rows": []}
        elif key == "row":
            cur["rows"].append([float(v) for v in vals])
        elif key in ("q", "r"):
            cur[key] = np.array([float(v) for v in vals], dtype=np.float32)
        elif key == "chunks":
            cur[key] = [int(v) for v in vals]
        elif key == "cost":
            cur[key] = float(vals[0])
        elif key == "end":
            cur[key] = int(vals[0])
    if cur:
        cases.append(cur)
    return cases


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_hand_worked_tables(oracle_mod, case):
    """Hand-computed tables from the Sec. 2.2 definition (tests/golden)."""
    q, r = case["q"], case["r"]
    if "chunks" in case:
        row = None
        pos = 0
        for k, size in enumerate(case["chunks"]):
            c, e, row = oracle_mod.dtw_f64(q[pos:pos + size], r, init_row=row, want_row=True)
            assert list(row) == case["rows"][k]
            pos += size
    else:
        D = oracle_mod.dtw_matrix_f64(q, r)
        assert D.tolist() == case["rows"]
        c, e = oracle_mod.dtw_f64(q, r)
    assert c == case["cost"] and e == case["end"]
    c32, e32 = oracle_mod.dtw_f32(q, r)
    assert float(c32) == case["cost"] and e32 == case["end"]


def _inputs(rng, n, m, kind):
    if kind == "normal":
        return (rng.standard_normal(n).astype(np.float32), rng.standard_normal(m).astype(np.float32))
    if kind == "dyadic":   # exact sums, many exact ties
        return W.dyadic_values(rng, n, -2, 2, 0.5), W.dyadic_values(rng, m, -2, 2, 0.5)
    if kind == "ints":     # heavy ties
        return (rng.integers(0, 3, n).astype(np.float32), rng.integers(0, 3, m).astype(np.float32))
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["normal", "dyadic", "ints"])
def test_brute_force_all_small_shapes(oracle_mod, kind):
    """Explicit enumeration of every warping path equals the recurrence
    exactly, cost and smallest end, for every n <= 5, m <= 7."""
    rng = np.random.default_rng(11 + len(kind))
    for n in range(1, 6):
        for m in range(1, 8):
            for _ in range(2):
                q, r = _inputs(rng, n, m, kind)
                bc, be, cnt = brute.brute_dtw(q, r)
                assert cnt > 0
                c, e = oracle_mod.dtw_f64(q, r)
                assert (c, e) == (bc, be), (n, m, q, r)


def test_brute_force_6x8(oracle_mod):
    rng = np.random.default_rng(68)
    for kind in ("normal", "ints"):
        q, r = _inputs(rng, 6, 8, kind)
        bc, be, cnt = brute.brute_dtw(q, r)
        assert (bc, be) == oracle_mod.dtw_f64(q, r)


def test_path_enumerator_counts():
    """The walker's path count for n = 1 is m(m+1)/2 (start s <= stop e in
    the single row), and for m = 1 it is 1 (straight down)."""
    for m in range(1, 9):
        assert brute.brute_dtw([0.0], [0.0] * m)[2] == m * (m + 1) // 2
    for n in range(1, 7):
        assert brute.brute_dtw([0.0] * n, [0.0])[2] == 1
        assert sum(1 for _ in brute.enumerate_paths(n, 1)) == 1


def _global_dtw(q, r):
    """Textbook global DTW (both ends fixed), written independently: the path
    must start at (0, 0) and end at (n-1, m-1)."""
    n, m = len(q), len(r)
    G = np.full((n, m), np.inf)
    for i in range(n):
        for j in range(m):
            c = abs(float(q[i]) - float(r[j]))
            if i == 0 and j == 0:
                G[i, j] = c
                continue
            best = np.inf
            if i > 0:
                best = min(best, G[i - 1, j])
            if j > 0:
                best = min(best, G[i, j - 1])
            if i > 0 and j > 0:
                best = min(best, G[i - 1, j - 1])
            G[i, j] = c + best
    return G[n - 1, m - 1]


@pytest.mark.parametrize("kind", ["normal", "ints"])
def test_min_over_windows_of_global_dtw(oracle_mod, kind):
    """Subsequence DTW = min over region windows [s, e] of global DTW of the
    query against r[s..e]; the end is the smallest e attaining it."""
    rng = np.random.default_rng(5)
    for _ in range(12):
        n, m = int(rng.integers(1, 7)), int(rng.integers(1, 10))
        q, r = _inputs(rng, n, m, kind)
        best, best_e = math.inf, -1
        for e in range(m):
            for s in range(e + 1):
                g = _global_dtw(q, r[s:e + 1])
                if g < best:
                    best, best_e = g, e
        assert oracle_mod.dtw_f64(q, r) == (best, best_e)


def test_single_event_is_nearest_level(oracle_mod):
    """n = 1: the cost is the distance to the nearest level and the end is
    the first index of it (numpy argmin returns the first minimum)."""
    rng = np.random.default_rng(1)
    for m in (1, 2, 7, 64, 1000):
        q = rng.standard_normal(1).astype(np.float32)
        r = rng.integers(-3, 4, m).astype(np.float32)  # ties on purpose
        d = np.abs(q.astype(np.float64)[0] - r.astype(np.float64))
        assert oracle_mod.dtw_f64(q, r) == (d.min(), int(np.argmin(d)))


def test_single_level_is_sum_of_deviations(oracle_mod):
    """m = 1: the only path goes straight down, so the cost is the sum of
    absolute deviations from r_0 (sequential sum), end 0; math.fsum bounds it."""
    rng = np.random.default_rng(2)
    for n in (1, 2, 5, 333):
        q = rng.standard_normal(n).astype(np.float32)
        r = rng.standard_normal(1).astype(np.float32)
        dev = [abs(float(x) - float(r[0])) for x in q]
        seq = 0.0
        for d in dev:
            seq = seq + d
        c, e = oracle_mod.dtw_f64(q, r)
        assert e == 0 and c == seq
        assert abs(c - math.fsum(dev)) <= 1e-12 * max(1.0, c)


def test_embedded_copy_with_dwell_costs_zero(oracle_mod):
    """A read that repeats each level of a region window (dwell, vertical
    steps) or skips repeated reference levels (horizontal steps) aligns at
    cost exactly 0, ending at the window's last level."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        m = int(rng.integers(20, 200))
        r = rng.standard_normal(m).astype(np.float32)  # distinct with probability 1
        s = int(rng.integers(0, m - 10))
        L = int(rng.integers(1, m - s))
        reps = rng.integers(1, 5, L)
        q = np.repeat(r[s:s + L], reps)
        assert oracle_mod.dtw_f64(q, r) == (0.0, s + L - 1)
        # reference dwell: repeat each region level, query is the plain window
        rr = np.repeat(r, rng.integers(1, 4, m))
        first = {}
        for j, v in enumerate(rr):
            first.setdefault(float(v), j)
        q2 = r[s:s + L]
        c2, e2 = oracle_mod.dtw_f64(q2, rr)
        assert c2 == 0.0 and e2 == first[float(q2[-1])] and rr[e2] == q2[-1]


def test_reversal_shift_scale(oracle_mod):
    """Exact symmetries on exactly-summable inputs: reversing both sequences
    keeps the path set (so the cost), adding one constant to both keeps every
    difference, scaling by 2 doubles every rounded operation exactly."""
    rng = np.random.default_rng(4)
    for _ in range(30):
        n, m = int(rng.integers(1, 40)), int(rng.integers(1, 60))
        q = W.dyadic_values(rng, n)
        r = W.dyadic_values(rng, m)
        c, e = oracle_mod.dtw_f64(q, r)
        assert oracle_mod.dtw_f64(q[::-1], r[::-1])[0] == c
        a = np.float32(0.75)
        assert oracle_mod.dtw_f64(q + a, r + a) == (c, e)
    for _ in range(10):
        q = rng.standard_normal(50).astype(np.float32)
        r = rng.standard_normal(80).astype(np.float32)
        c, e = oracle_mod.dtw_f64(q, r)
        c2, e2 = oracle_mod.dtw_f64(2 * q, 2 * r)
        assert (c2, e2) == (2 * c, e)
        cr = oracle_mod.dtw_f64(q[::-1], r[::-1])[0]
        assert abs(cr - c) <= 1e-12 * c


def test_table_invariants(oracle_mod):
    """D >= c >= 0; each row's minimum never decreases (every cell extends a
    path through the previous row); the rolling-row result equals the full
    table's last row; the cost lies between the sum of per-row minimum costs
    and the cost of one explicit path."""
    rng = np.random.default_rng(6)
    for _ in range(20):
        n, m = int(rng.integers(1, 30)), int(rng.integers(1, 50))
        q = rng.standard_normal(n).astype(np.float32)
        r = rng.standard_normal(m).astype(np.float32)
        D = oracle_mod.dtw_matrix_f64(q, r)
        cost = np.abs(q.astype(np.float64)[:, None] - r.astype(np.float64)[None, :])
        assert (D >= cost).all() and (cost >= 0).all()
        rowmin = D.min(axis=1)
        assert (np.diff(rowmin) >= 0).all()
        c, e, last = oracle_mod.dtw_f64(q, r, want_row=True)
        assert np.array_equal(last, D[-1]) and c == D[-1].min() and e == int(np.argmin(D[-1]))
        lower = cost.min(axis=1).sum()
        path = sum(cost[i, min(i, m - 1)] for i in range(n))  # a valid staircase path
        assert lower <= c * (1 + 1e-12) and c <= path * (1 + 1e-12)


def test_chunked_equals_whole(oracle_mod):
    """Carrying the last row across chunks (Read Until streaming) gives the
    same rows, cost and end as aligning the whole prefix at once."""
    rng = np.random.default_rng(7)
    for _ in range(10):
        n, m = int(rng.integers(2, 300)), int(rng.integers(1, 400))
        q = rng.standard_normal(n).astype(np.float32)
        r = rng.standard_normal(m).astype(np.float32)
        cuts = sorted(set(rng.integers(1, n, size=3).tolist()))
        bounds = [0] + cuts + [n]
        row64 = row32 = None
        for a, b in zip(bounds[:-1], bounds[1:]):
            c64, e64, row64 = oracle_mod.dtw_f64(q[a:b], r, init_row=row64, want_row=True)
            c32, e32, row32 = oracle_mod.dtw_f32(q[a:b], r, init_row=row32, want_row=True)
            w64 = oracle_mod.dtw_f64(q[:b], r, want_row=True)
            w32 = oracle_mod.dtw_f32(q[:b], r, want_row=True)
            assert (c64, e64) == w64[:2] and np.array_equal(row64, w64[2])
            assert (c32, e32) == w32[:2] and np.array_equal(row32, w32[2])


def test_float_equals_double_on_exact_inputs(oracle_mod):
    """With quarter-integer inputs every partial sum is exact in float, so
    the float recurrence must equal the double one bit for bit, ties too."""
    rng = np.random.default_rng(8)
    for _ in range(30):
        n, m = int(rng.integers(1, 120)), int(rng.integers(1, 200))
        q = W.dyadic_values(rng, n)
        r = W.dyadic_values(rng, m)
        c64, e64 = oracle_mod.dtw_f64(q, r)
        c32, e32 = oracle_mod.dtw_f32(q, r)
        assert float(c32) == c64 and e32 == e64


def test_float_error_within_rounding_bound(oracle_mod):
    """On real-valued inputs the float result is within the forward error
    bound of (n + m) roundings of its own magnitude."""
    rng = np.random.default_rng(9)
    for _ in range(10):
        n, m = int(rng.integers(100, 600)), int(rng.integers(100, 900))
        q = rng.standard_normal(n).astype(np.float32)
        r = rng.standard_normal(m).astype(np.float32)
        c64, _ = oracle_mod.dtw_f64(q, r)
        c32, _ = oracle_mod.dtw_f32(q, r)
        assert abs(float(c32) - c64) <= (n + m) * 2.0 ** -23 * c64 + 1e-30


def test_degenerate_sizes(oracle_mod):
    r = np.array([1.0, 2.0], np.float32)
    assert oracle_mod.dtw_f64(np.zeros(0, np.float32), r) == (0.0, -1)
    c, e = oracle_mod.dtw_f64(np.ones(3, np.float32), np.zeros(0, np.float32))
    assert c == math.inf and e == -1
    assert oracle_mod.dtw_f32(np.zeros(0, np.float32), np.zeros(0, np.float32)) == (0.0, -1)


def test_batch_matches_single_and_threads(oracle_mod):
    rng = np.random.default_rng(10)
    b = W.random_pairs(rng, 37, (0, 70), (0, 90))
    s1, e1, used1 = oracle_mod.dtw_batch_f64(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, threads=1)
    s8, e8, used8 = oracle_mod.dtw_batch_f64(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, threads=8)
    assert used1 == 1 and used8 >= 1
    assert np.array_equal(s1, s8) and np.array_equal(e1, e8)
    for p in range(b.n_pairs):
        q = b.q[b.q_off[p]:b.q_off[p] + b.q_len[p]]
        r = b.r[b.r_off[p]:b.r_off[p] + b.r_len[p]]
        c, e = oracle_mod.dtw_f64(q, r)
        assert (s1[p] == c or (math.isinf(c) and math.isinf(s1[p]))) and e1[p] == e
    f32, fe, _ = oracle_mod.dtw_batch_f32(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, threads=4)
    for p in range(b.n_pairs):
        q = b.q[b.q_off[p]:b.q_off[p] + b.q_len[p]]
        r = b.r[b.r_off[p]:b.r_off[p] + b.r_len[p]]
        c, e = oracle_mod.dtw_f32(q, r)
        assert (f32[p] == c or (math.isinf(c) and math.isinf(f32[p]))) and fe[p] == e


def test_decision_worked_examples(oracle_mod):
    """Sec. 2.3: Score = B_Match * N_Read - C_DTW; the highest-scoring
    candidate is mapped iff its score is at least the threshold (0.4 and 20,
    Sec. 3.1.5).  Hand-computed: N = 100 gives a bonus of 40."""
    cost = np.array([25.0, 19.5, 20.0, 30.0, 0.0, np.inf], np.float32)
    cand_off = np.array([0, 3, 4, 5, 6])
    cand_cnt = np.array([3, 1, 1, 1, 0])
    n_events = np.array([100, 100, 50, 10, 10])
    best, score, mapped = oracle_mod.decide(cost, cand_off, cand_cnt, n_events)
    # read 0: scores 15, 20.5, 20 -> pair 1, 20.5 >= 20 -> mapped
    # read 1: 40 - 30 = 10 -> not mapped; read 2: 0.4*50 - 0 = 20 -> mapped (at threshold)
    # read 3: cost +inf -> score -inf, not mapped; read 4: no candidates
    assert best.tolist() == [1, 3, 4, 5, -1]
    assert score[0] == 0.4 * 100 - 19.5 and score[2] == 0.4 * 50
    assert score[3] == -np.inf and score[4] == -np.inf
    assert mapped.tolist() == [1, 0, 1, 0, 0]
    # equal scores: the smaller pair index wins
    b2, _, _ = oracle_mod.decide(np.array([5.0, 5.0], np.float32), [0], [2], [100])
    assert b2.tolist() == [0]


def test_decision_skips_nan_sentinels(oracle_mod):
    """A NaN cost is the sentinel of a pair that was not aligned: it is not a
    candidate.  Hand-computed, N = 100 (bonus 40): read 0 has the sentinel
    first and a mapping candidate (40 - 10 = 30) after it; read 1 has only
    sentinels (no candidate: -1, -inf); read 2 has a sentinel between two
    real candidates (scores 15 and 25)."""
    nan = np.float32(np.nan)
    cost = np.array([nan, 10.0, nan, nan, 25.0, nan, 15.0], np.float32)
    best, score, mapped = oracle_mod.decide(cost, [0, 2, 4], [2, 2, 3], [100, 100, 100])
    assert best.tolist() == [1, -1, 6]
    assert score.tolist() == [30.0, -np.inf, 25.0]
    assert mapped.tolist() == [1, 0, 1]
