"""Pins of the oracle's anchor-guided alignment (Sec. 2.4.2) to facts that do
not come from the oracle itself: path enumeration, closed forms of one-row
and one-column gaps, the relation to subsequence DTW, exact arithmetic, and
hand-worked chain sums and decisions."""
import math

import numpy as np
import pytest

from oracle import brute
from paper_2310_05037_amd import workloads as W


def _inputs(rng, n, m, kind):
    if kind == "ints":
        return (rng.integers(-3, 4, size=n).astype(np.float32), rng.integers(-3, 4, size=m).astype(np.float32))
    return rng.standard_normal(n).astype(np.float32), rng.standard_normal(m).astype(np.float32)


def test_global_path_counts_are_delannoy_numbers():
    """Monotone lattice paths from (0,0) to (a,b) with unit steps E, N, NE
    number the Delannoy numbers: D(1,1)=3, D(2,2)=13, D(2,3)=25, D(3,3)=63,
    D(4,5)=681."""
    for (a, b), d in {(1, 1): 3, (2, 2): 13, (2, 3): 25, (3, 3): 63, (4, 5): 681, (0, 4): 1}.items():
        assert brute.brute_global_dtw([0.0] * (a + 1), [0.0] * (b + 1))[1] == d


@pytest.mark.parametrize("kind", ["normal", "ints"])
def test_global_matches_brute_force_all_small_shapes(oracle_mod, kind):
    """Every shape up to 5 x 6: the table equals the cheapest enumerated path
    exactly (a rounded addition is monotone, so the table's minimum of
    rounded path sums is the enumeration's)."""
    rng = np.random.default_rng(11)
    for n in range(1, 6):
        for m in range(1, 7):
            q, r = _inputs(rng, n, m, kind)
            cost, _ = brute.brute_global_dtw(q, r)
            assert oracle_mod.dtw_global_f64(q, r) == cost, (n, m)


def test_global_single_row_and_column_are_sums(oracle_mod):
    """n = 1: the path must cross every level of the gap, so the cost is
    sum_j |q_0 - r_j|; m = 1: sum_i |q_i - r_0|."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        m = int(rng.integers(1, 30))
        q = rng.standard_normal(1).astype(np.float32)
        r = rng.standard_normal(m).astype(np.float32)
        exp = math.fsum(abs(float(q[0]) - float(x)) for x in r)
        assert oracle_mod.dtw_global_f64(q, r) == pytest.approx(exp, rel=1e-14, abs=0)
        qq = rng.standard_normal(m).astype(np.float32)
        exp2 = math.fsum(abs(float(x) - float(q[0])) for x in qq)
        assert oracle_mod.dtw_global_f64(qq, q) == pytest.approx(exp2, rel=1e-14, abs=0)


def test_global_zero_on_a_warped_copy(oracle_mod):
    """Levels repeated by a dwell of at least one event each, aligned against
    the levels themselves, cost 0; one changed event costs exactly its
    deviation when it stays closest to its own level."""
    rng = np.random.default_rng(4)
    for _ in range(10):
        m = int(rng.integers(1, 25))
        r = (rng.integers(-40, 41, size=m) * 0.25).astype(np.float32)
        q = np.repeat(r, rng.integers(1, 4, size=m))
        assert oracle_mod.dtw_global_f64(q, r) == 0.0
        assert oracle_mod.dtw_global_f32(q, r) == 0.0


def test_global_is_subsequence_with_fixed_ends(oracle_mod):
    """Global DTW never costs less than subsequence DTW of the same pair,
    and the minimum of global DTW over all region windows [s, e] is the
    subsequence cost (the windows are exactly the free start and end)."""
    rng = np.random.default_rng(6)
    for _ in range(25):
        n, m = int(rng.integers(1, 7)), int(rng.integers(1, 9))
        q, r = _inputs(rng, n, m, "normal")
        sub, _ = oracle_mod.dtw_f64(q, r)
        assert oracle_mod.dtw_global_f64(q, r) >= sub
        best = min(oracle_mod.dtw_global_f64(q, r[s:e + 1]) for e in range(m) for s in range(e + 1))
        assert best == sub


def test_global_degenerate_sizes(oracle_mod):
    """Anchors touching diagonally: 0.  Events without levels or levels
    without events: no path through the gap's cells, +inf."""
    for f in (oracle_mod.dtw_global_f64, oracle_mod.dtw_global_f32):
        assert f([], []) == 0.0
        assert f([1.0], []) == math.inf and f([], [1.0, 2.0]) == math.inf
        assert f([1.5], [0.5]) == 1.0


def test_global_float_equals_double_on_exact_inputs(oracle_mod):
    rng = np.random.default_rng(8)
    for _ in range(20):
        n, m = int(rng.integers(1, 60)), int(rng.integers(1, 60))
        q, r = W.dyadic_values(rng, n), W.dyadic_values(rng, m)
        assert float(oracle_mod.dtw_global_f32(q, r)) == oracle_mod.dtw_global_f64(q, r)


def test_global_float_error_within_rounding_bound(oracle_mod):
    """Every cell adds one rounding of relative size 2^-24 to the path sum,
    so a float result is within (n + m) 2^-24 of the double one (relative)."""
    rng = np.random.default_rng(9)
    for _ in range(10):
        n, m = int(rng.integers(50, 300)), int(rng.integers(20, 100))
        q, r = _inputs(rng, n, m, "normal")
        d = oracle_mod.dtw_global_f64(q, r)
        f = float(oracle_mod.dtw_global_f32(q, r))
        assert abs(f - d) <= (n + m) * 2.0 ** -24 * d + 1e-30


def test_global_batch_matches_single(oracle_mod):
    rng = np.random.default_rng(10)
    b = W.random_pairs(rng, 50, (0, 40), (0, 30))
    for fb, fs in ((oracle_mod.dtw_global_batch_f64, oracle_mod.dtw_global_f64),
                   (oracle_mod.dtw_global_batch_f32, oracle_mod.dtw_global_f32)):
        out, _ = fb(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, threads=3)
        for p in range(b.n_pairs):
            exp = fs(b.q[b.q_off[p]:b.q_off[p] + b.q_len[p]], b.r[b.r_off[p]:b.r_off[p] + b.r_len[p]])
            assert out[p] == exp or (math.isinf(out[p]) and math.isinf(exp))


def test_chain_cost_sums_in_gap_order(oracle_mod):
    """A chain costs the sum of its gaps, added in gap order: in float,
    (2^24 + 1) + 1 rounds back to 2^24 each time, while 1 + 1 + 2^24 would
    give 2^24 + 2.  A chain without gaps costs 0; an out-of-range gap range
    gives NaN."""
    g = np.array([2.0 ** 24, 1.0, 1.0, 1.5, 2.25, np.inf], np.float32)
    cost = oracle_mod.chain_costs(g, [0, 3, 5, 6, 4], [3, 2, 1, 0, 3])
    assert cost.dtype == np.float32
    assert cost[0] == np.float32(2.0 ** 24) and cost[1] == np.float32(3.75)
    assert cost[2] == np.inf and cost[3] == 0.0 and np.isnan(cost[4])
    g64 = g.astype(np.float64)
    assert oracle_mod.chain_costs(g64, [0], [3])[0] == 2.0 ** 24 + 2


def test_decide_chains_worked_example(oracle_mod):
    """Score = 0.4 * (events the chain aligns) - chain cost; highest wins,
    smallest index on ties, mapped iff >= 20.  Hand-computed."""
    cost = np.array([10.0, 5.0, 30.0, 0.0, 1.0, 1.0], np.float32)
    events = np.array([100, 50, 100, 40, 60, 60])
    best, score, mapped = oracle_mod.decide_chains(cost, events, [0, 2, 3, 4, 6], [2, 1, 1, 2, 0])
    # read 0: 40-10=30 vs 20-5=15 -> chain 0, mapped; read 1: 40-30=10 -> not mapped
    # read 2: 16-0=16 -> not mapped; read 3: 23 vs 23 -> chain 4 (smaller index); read 4: none
    assert best.tolist() == [0, 2, 3, 4, -1]
    assert score[0] == 30.0 and score[2] == pytest.approx(16.0) and score[3] == pytest.approx(23.0)
    assert mapped.tolist() == [1, 0, 0, 1, 0]


def test_decide_chains_skips_nan_costs(oracle_mod):
    """A chain whose cost is NaN (its gap range left the gap array) is no
    candidate: the next chain of the read still wins.  Hand-computed: read 0
    has a NaN chain then 0.4*100 - 10 = 30; read 1 has only a NaN chain."""
    cost = np.array([np.nan, 10.0, np.nan], np.float32)
    best, score, mapped = oracle_mod.decide_chains(cost, [100, 100, 100], [0, 2], [2, 1])
    assert best.tolist() == [1, -1] and score.tolist() == [30.0, -np.inf] and mapped.tolist() == [1, 0]


def test_anchored_workload_structure():
    """Every gap lies inside q and r and is empty on both sides or on
    neither; a chain's gaps advance through the read and the reference;
    the true chain's gaps cost far less per event than decoy gaps."""
    a = W.anchored_chains(600, ref_bases=1_000_000)
    assert a.n_chains == 600 and int(a.cand_cnt.sum()) == 600
    assert ((a.gap_q_len == 0) == (a.gap_r_len == 0)).all()
    assert (a.gap_q_off >= 0).all() and (a.gap_q_off + a.gap_q_len <= len(a.q)).all()
    assert (a.gap_r_off >= 0).all() and (a.gap_r_off + a.gap_r_len <= len(a.r)).all()
    for c in range(a.n_chains):
        g0, cnt = int(a.chain_gap_off[c]), int(a.chain_gap_cnt[c])
        qe = a.gap_q_off[g0:g0 + cnt] + a.gap_q_len[g0:g0 + cnt]
        re = a.gap_r_off[g0:g0 + cnt] + a.gap_r_len[g0:g0 + cnt]
        assert (a.gap_q_off[g0 + 1:g0 + cnt] >= qe[:-1]).all() and (a.gap_r_off[g0 + 1:g0 + cnt] >= re[:-1]).all()
        assert int(a.gap_q_len[g0:g0 + cnt].sum()) <= int(a.chain_events[c])
    from oracle import oracle
    g, _ = oracle.dtw_global_batch_f64(a.q, a.gap_q_off, a.gap_q_len, a.r, a.gap_r_off, a.gap_r_len)
    is_true = np.zeros(a.n_chains, bool)
    is_true[a.true_chain] = True
    gap_true = np.repeat(is_true, a.chain_gap_cnt)
    per_ev = g / np.maximum(a.gap_q_len, 1)
    assert np.median(per_ev[gap_true]) < 0.5 * np.median(per_ev[~gap_true])
