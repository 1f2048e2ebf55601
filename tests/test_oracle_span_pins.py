"""Pins of the oracle's alignment start (the path's first region column) to
facts that do not come from the oracle itself: explicit path enumeration,
the global cost of the aligned interval, single-event queries, embedded
copies, exact arithmetic."""
import math

import numpy as np
import pytest

from oracle import brute
from paper_2310_05037_amd import workloads as W


def _inputs(rng, n, m, kind):
    if kind == "ints":
        return (rng.integers(-3, 4, size=n).astype(np.float32), rng.integers(-3, 4, size=m).astype(np.float32))
    return rng.standard_normal(n).astype(np.float32), rng.standard_normal(m).astype(np.float32)


@pytest.mark.parametrize("kind", ["normal", "ints"])
def test_span_matches_brute_force_all_small_shapes(oracle_mod, kind):
    """Every shape up to 5 x 6: cost, end (smallest final column among the
    cheapest paths) and start (largest first column among the cheapest
    paths ending there) equal the enumeration; integer inputs make ties
    common and every sum exact."""
    rng = np.random.default_rng(21)
    for n in range(1, 6):
        for m in range(1, 7):
            for _ in range(2):
                q, r = _inputs(rng, n, m, kind)
                assert oracle_mod.dtw_span_f64(q, r) == brute.brute_span(q, r), (n, m, q, r)


def test_span_interval_has_the_global_cost(oracle_mod):
    """The aligned interval [start, end] of the region, aligned globally,
    costs exactly C_DTW (integer inputs: every sum exact), and start <= end."""
    rng = np.random.default_rng(22)
    for _ in range(60):
        n, m = int(rng.integers(1, 12)), int(rng.integers(1, 30))
        q, r = _inputs(rng, n, m, "ints")
        c, e, s = oracle_mod.dtw_span_f64(q, r)
        assert 0 <= s <= e < m
        assert oracle_mod.dtw_global_f64(q, r[s:e + 1]) == c
        # no later start reaches the same cost with the same end
        for s2 in range(s + 1, e + 1):
            assert oracle_mod.dtw_global_f64(q, r[s2:e + 1]) > c


def test_span_single_event_is_one_cell(oracle_mod):
    """n = 1: any path is a run of row 0 whose cost includes |q - r_end|, so
    the latest start is the end itself."""
    rng = np.random.default_rng(23)
    for _ in range(20):
        m = int(rng.integers(1, 40))
        q = rng.standard_normal(1).astype(np.float32)
        r = rng.standard_normal(m).astype(np.float32)
        c, e, s = oracle_mod.dtw_span_f64(q, r)
        assert s == e == int(np.argmin(np.abs(r.astype(np.float64) - float(q[0]))))


def test_span_of_an_embedded_copy(oracle_mod):
    """A read made of levels a .. b of the region (each repeated by a dwell)
    aligns at cost 0 from a to b (levels distinct, so the zero-cost path is
    unique)."""
    rng = np.random.default_rng(24)
    for _ in range(15):
        m = int(rng.integers(10, 60))
        r = rng.standard_normal(m).astype(np.float32)
        a = int(rng.integers(0, m - 3))
        b = int(rng.integers(a + 1, m))
        q = np.repeat(r[a:b + 1], rng.integers(1, 4, size=b - a + 1))
        for f in (oracle_mod.dtw_span_f64, oracle_mod.dtw_span_f32):
            c, e, s = f(q, r)
            assert c == 0 and (s, e) == (a, b)


def test_span_float_equals_double_on_exact_inputs(oracle_mod):
    rng = np.random.default_rng(25)
    for _ in range(30):
        n, m = int(rng.integers(1, 40)), int(rng.integers(1, 80))
        q, r = W.dyadic_values(rng, n), W.dyadic_values(rng, m)
        c64, e64, s64 = oracle_mod.dtw_span_f64(q, r)
        c32, e32, s32 = oracle_mod.dtw_span_f32(q, r)
        assert float(c32) == c64 and (e32, s32) == (e64, s64)


def test_span_degenerate_and_batch(oracle_mod):
    assert oracle_mod.dtw_span_f64([], [1.0]) == (0.0, -1, -1)
    c, e, s = oracle_mod.dtw_span_f64([1.0], [])
    assert math.isinf(c) and (e, s) == (-1, -1)
    rng = np.random.default_rng(26)
    b = W.random_pairs(rng, 40, (0, 30), (0, 50))
    for fb, fs in ((oracle_mod.dtw_span_batch_f64, oracle_mod.dtw_span_f64),
                   (oracle_mod.dtw_span_batch_f32, oracle_mod.dtw_span_f32)):
        sc, en, st = fb(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, threads=3)
        for p in range(b.n_pairs):
            c, e, s = fs(b.q[b.q_off[p]:b.q_off[p] + b.q_len[p]], b.r[b.r_off[p]:b.r_off[p] + b.r_len[p]])
            assert (sc[p] == c or (math.isinf(sc[p]) and math.isinf(c))) and (en[p], st[p]) == (e, s)
