"""Pins of the warping-path oracle (Sec. 2.4: the alignment path as an
optional output) against facts it does not compute itself: brute-force path
enumeration with the same tie rule, the path's own cost, the shape of a
monotone path, and the subsequence score it realises."""
import math

import numpy as np
import pytest

from oracle import brute, oracle


@pytest.fixture(scope="module")
def oracle_mod():
    oracle.build(force=False)
    return oracle


def _check_shape(lo, hi, start, end):
    n = len(lo)
    assert lo[0] == start and hi[n - 1] == end
    for i in range(n):
        assert lo[i] <= hi[i]
        if i + 1 < n:
            assert lo[i + 1] in (hi[i], hi[i] + 1)


def _path_cost(q, r, lo, hi):
    return math.fsum(abs(float(q[i]) - float(r[j])) for i in range(len(q)) for j in range(lo[i], hi[i] + 1))


@pytest.mark.parametrize("kind", ["int", "quarter"])
def test_path_matches_brute_force_tie_rule(oracle_mod, kind):
    """Small integer (or quarter-step) inputs with many equal costs: the
    oracle's path is exactly the enumerated optimal path whose backward moves
    come first in the order north-west, north, west."""
    rng = np.random.default_rng(71 if kind == "int" else 72)
    for _ in range(120):
        n = int(rng.integers(1, 6))
        m = int(rng.integers(1, 8))
        if kind == "int":
            q = rng.integers(-2, 3, n).astype(np.float32)
            r = rng.integers(-2, 3, m).astype(np.float32)
        else:
            q = (rng.integers(-8, 9, n) * 0.25).astype(np.float32)
            r = (rng.integers(-8, 9, m) * 0.25).astype(np.float32)
        c, e, s, g, lo, hi = oracle_mod.dtw_path_f64(q, r)
        bc, blo, bhi = brute.brute_path(q, r, s, e)
        assert g == bc == c
        assert list(lo) == blo and list(hi) == bhi


def test_path_realises_the_score(oracle_mod):
    """Normal inputs: the path is monotone from (0, start) to (n-1, end), its
    cells' costs add up to C_DTW, and the float path is the float table's."""
    rng = np.random.default_rng(73)
    for _ in range(60):
        n = int(rng.integers(1, 60))
        m = int(rng.integers(1, 90))
        q = rng.standard_normal(n).astype(np.float32)
        r = rng.standard_normal(m).astype(np.float32)
        c, e, s, g, lo, hi = oracle_mod.dtw_path_f64(q, r)
        _check_shape(lo, hi, s, e)
        assert g == pytest.approx(c, rel=1e-12, abs=1e-12)
        assert _path_cost(q, r, lo, hi) == pytest.approx(c, rel=1e-12, abs=1e-12)
        c32, e32, s32, g32, lo32, hi32 = oracle_mod.dtw_path_f32(q, r)
        _check_shape(lo32, hi32, s32, e32)
        assert abs(float(g32) - c) <= 1e-4 * abs(c) + 1e-6


def test_path_special_cases(oracle_mod):
    """One event: a single cell at the nearest level.  One level: every
    event on it.  An embedded copy with dwell: each event on its own level.
    Empty query or region: no path."""
    rng = np.random.default_rng(74)
    r = rng.standard_normal(30).astype(np.float32)
    q = np.array([r[17] + 0.01], dtype=np.float32)
    c, e, s, g, lo, hi = oracle_mod.dtw_path_f64(q, r)
    assert (s, e, list(lo), list(hi)) == (17, 17, [17], [17])
    q = rng.standard_normal(9).astype(np.float32)
    c, e, s, g, lo, hi = oracle_mod.dtw_path_f64(q, r[4:5])
    assert list(lo) == [0] * 9 and list(hi) == [0] * 9
    dwell = [1, 3, 2, 1, 4, 2]
    q = np.repeat(r[10:16], dwell).astype(np.float32)
    c, e, s, g, lo, hi = oracle_mod.dtw_path_f64(q, r)
    assert c == 0.0 and (s, e) == (10, 15)
    assert list(lo) == list(np.repeat(np.arange(10, 16), dwell)) and list(lo) == list(hi)
    for qq, rr in ((np.zeros(0, np.float32), r), (q, np.zeros(0, np.float32))):
        _, e, s, _, lo, hi = oracle_mod.dtw_path_f64(qq, rr)
        assert e == -1 and s == -1 and (lo == -1).all() and (hi == -1).all()


def test_path_float_equals_double_on_exact_inputs(oracle_mod):
    """Quarter-step inputs keep every sum exact in float: the float path
    (start from the float reverse pass, directions from the float table) is
    the double one, ties and all."""
    rng = np.random.default_rng(75)
    for _ in range(80):
        n = int(rng.integers(1, 50))
        m = int(rng.integers(1, 70))
        q = (rng.integers(-8, 9, n) * 0.25).astype(np.float32)
        r = (rng.integers(-8, 9, m) * 0.25).astype(np.float32)
        c, e, s, g, lo, hi = oracle_mod.dtw_path_f64(q, r)
        c32, e32, s32, g32, lo32, hi32 = oracle_mod.dtw_path_f32(q, r)
        assert float(c32) == c and (e32, s32) == (e, s) and float(g32) == g
        assert list(lo32) == list(lo) and list(hi32) == list(hi)
