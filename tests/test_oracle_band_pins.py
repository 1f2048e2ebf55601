"""Pins of the oracle's banded DTW (Sec. 2.4.3) to facts that do not come
from the oracle itself: explicit enumeration of the paths inside the band,
the full band equalling plain subsequence DTW, wider bands never costing
more, the diagonal band as a sum of deviations, exact arithmetic."""
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
def test_band_matches_brute_force(oracle_mod, kind):
    """Every shape up to 6 x 6 and every half-width up to m: the table equals
    the cheapest path that stays in the band, and its smallest end."""
    rng = np.random.default_rng(31)
    for n in range(1, 7):
        for m in range(1, 7):
            q, r = _inputs(rng, n, m, kind)
            for w in range(0, m + 1):
                assert oracle_mod.dtw_band_f64(q, r, w) == brute.brute_band(q, r, w), (n, m, w)


def test_full_band_is_plain_subsequence_dtw(oracle_mod):
    """w >= m-1 admits every cell: the plain recurrence's cost and end, bit
    for bit in both precisions."""
    rng = np.random.default_rng(32)
    for _ in range(30):
        n, m = int(rng.integers(1, 60)), int(rng.integers(1, 60))
        q, r = _inputs(rng, n, m, "normal")
        for w in (m - 1, m, 3 * m):
            assert oracle_mod.dtw_band_f64(q, r, w) == oracle_mod.dtw_f64(q, r)
            c32, e32 = oracle_mod.dtw_band_f32(q, r, w)
            p32, pe32 = oracle_mod.dtw_f32(q, r)
            assert c32.view(np.uint32) == np.float32(p32).view(np.uint32) and e32 == pe32


def test_wider_band_never_costs_more(oracle_mod):
    """A wider band admits a superset of paths; rounded addition is monotone,
    so the float table is monotone too."""
    rng = np.random.default_rng(33)
    for _ in range(30):
        n, m = int(rng.integers(2, 80)), int(rng.integers(2, 80))
        q, r = _inputs(rng, n, m, "normal")
        prev64, prev32 = math.inf, np.float32(np.inf)
        for w in range(0, m + 1, max(1, m // 7)):
            c64, _ = oracle_mod.dtw_band_f64(q, r, w)
            c32, _ = oracle_mod.dtw_band_f32(q, r, w)
            assert c64 <= prev64 and c32 <= prev32
            prev64, prev32 = c64, c32


def test_diagonal_band_is_a_sum_of_deviations(oracle_mod):
    """n == m and w == 0: the only path is the diagonal, cost sum |q_i - r_i|,
    end m-1.  m == 2n and w == 0: cells (i, 2i) are not connected, +inf."""
    rng = np.random.default_rng(34)
    for _ in range(20):
        n = int(rng.integers(1, 40))
        q, r = _inputs(rng, n, n, "normal")
        c, e = oracle_mod.dtw_band_f64(q, r, 0)
        assert c == pytest.approx(math.fsum(abs(float(a) - float(b)) for a, b in zip(q, r)), rel=1e-14) and e == n - 1
        if n >= 2:
            q2, r2 = _inputs(rng, n, 2 * n, "normal")
            assert oracle_mod.dtw_band_f64(q2, r2, 0) == (math.inf, -1)


def test_band_single_event_and_degenerate(oracle_mod):
    """n = 1: row 0's band is columns 0 .. min(w, m-1): the nearest level
    among them."""
    rng = np.random.default_rng(35)
    for _ in range(20):
        m, w = int(rng.integers(1, 30)), int(rng.integers(0, 10))
        q = rng.standard_normal(1).astype(np.float32)
        r = rng.standard_normal(m).astype(np.float32)
        d = np.abs(r[:min(w, m - 1) + 1].astype(np.float64) - float(q[0]))
        assert oracle_mod.dtw_band_f64(q, r, w) == (float(d.min()), int(np.argmin(d)))
    assert oracle_mod.dtw_band_f64([], [1.0], 3) == (0.0, -1)
    c, e = oracle_mod.dtw_band_f64([1.0], [], 3)
    assert math.isinf(c) and e == -1


def test_band_float_equals_double_on_exact_inputs_and_batch(oracle_mod):
    rng = np.random.default_rng(36)
    for _ in range(20):
        n, m = int(rng.integers(1, 60)), int(rng.integers(1, 60))
        q, r = W.dyadic_values(rng, n), W.dyadic_values(rng, m)
        w = int(rng.integers(0, m + 1))
        c64, e64 = oracle_mod.dtw_band_f64(q, r, w)
        c32, e32 = oracle_mod.dtw_band_f32(q, r, w)
        assert (float(c32) == c64 or (math.isinf(c64) and math.isinf(c32))) and e32 == e64
    b = W.random_pairs(rng, 40, (0, 40), (0, 40))
    band = rng.integers(0, 20, size=b.n_pairs).astype(np.int32)
    for fb, fs in ((oracle_mod.dtw_band_batch_f64, oracle_mod.dtw_band_f64),
                   (oracle_mod.dtw_band_batch_f32, oracle_mod.dtw_band_f32)):
        sc, en = fb(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, band, threads=3)
        for p in range(b.n_pairs):
            c, e = fs(b.q[b.q_off[p]:b.q_off[p] + b.q_len[p]], b.r[b.r_off[p]:b.r_off[p] + b.r_len[p]], band[p])
            assert (sc[p] == c or (math.isinf(sc[p]) and math.isinf(c))) and en[p] == e
