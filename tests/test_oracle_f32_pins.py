"""Pins of the oracle's float32 instantiations to explicit path enumeration
in float32 (oracle/brute.py with f32=True).

The float functions are the bitwise reference of every GPU parity test.
Rounded addition is monotone, so on any input the float table holds the
smallest float path sum, each path summed cell by cell in float32 in path
order.  The enumeration computes that sum independently of the table, so
these tests hold on ordinary normal inputs, not only on exactly summable
ones: every shape up to 5 x 7 and 6 x 8, for plain, global, banded,
start-of-alignment and warping-path DTW (Sec. 2.2, 2.4, 2.4.2, 2.4.3).
"""
import numpy as np
import pytest

from oracle import brute

SHAPES = [(n, m) for n in range(1, 6) for m in range(1, 8)] + [(6, 8)]


def _bits(x) -> int:
    return int(np.float32(x).view(np.uint32))


def _same(a, b) -> bool:
    """Bit-identical float32 values (+inf included)."""
    return _bits(a) == _bits(b)


def _normal(rng, n, m):
    # Distinct, non-dyadic values: the differences and sums round.
    return rng.standard_normal(n).astype(np.float32), rng.standard_normal(m).astype(np.float32)


def _cases(seed, per_shape=2):
    rng = np.random.default_rng(seed)
    for n, m in SHAPES:
        for _ in range(per_shape):
            yield (n, m) + _normal(rng, n, m)


def test_f32_subsequence_matches_float_enumeration(oracle_mod):
    for n, m, q, r in _cases(101):
        bc, be, _ = brute.brute_dtw(q, r, f32=True)
        c, e = oracle_mod.dtw_f32(q, r)
        assert _same(c, bc) and e == be, (n, m, q, r, c, bc)


def test_f32_global_matches_float_enumeration(oracle_mod):
    for n, m, q, r in _cases(102):
        bc, _ = brute.brute_global_dtw(q, r, f32=True)
        assert _same(oracle_mod.dtw_global_f32(q, r), bc), (n, m, q, r)


def test_f32_band_matches_float_enumeration(oracle_mod):
    for n, m, q, r in _cases(103, per_shape=1):
        for w in range(0, m + 1):
            bc, be = brute.brute_band(q, r, w, f32=True)
            c, e = oracle_mod.dtw_band_f32(q, r, w)
            assert _same(c, bc) and e == be, (n, m, w, q, r)


def test_f32_span_matches_float_enumeration(oracle_mod):
    for n, m, q, r in _cases(104):
        bc, be, bs = brute.brute_span(q, r, f32=True)
        c, e, s = oracle_mod.dtw_span_f32(q, r)
        assert _same(c, bc) and e == be and s == bs, (n, m, q, r, (c, e, s), (bc, be, bs))


def test_f32_path_matches_float_enumeration(oracle_mod):
    for n, m, q, r in _cases(105):
        c, e, s, g, lo, hi = oracle_mod.dtw_path_f32(q, r)
        bg, blo, bhi = brute.brute_path_f32(q, r, s, e)
        assert _same(g, bg), (n, m, q, r)
        assert list(lo) == blo and list(hi) == bhi, (n, m, q, r)


def _double_intermediate_f32(q, r):
    """A plausible mistake in a float recurrence: the table kept in double
    and rounded to float only at the end.  Used only to show that the
    enumeration tells it apart from a true float table."""
    n, m = len(q), len(r)
    prev = [0.0] * (m + 1)
    for i in range(n):
        cur = [np.inf] * (m + 1)
        for j in range(m):
            c = abs(float(q[i]) - float(r[j]))
            cur[j + 1] = c + min(prev[j], prev[j + 1], cur[j])
        prev = cur
    row = prev[1:]
    e = int(np.argmin(row))
    return np.float32(row[e]), e


def test_enumeration_rejects_double_intermediates():
    """The float pin has teeth: on the same shapes the double-intermediate
    recurrence disagrees with the float enumeration on many cases, so an
    oracle that made that mistake would fail the tests above."""
    differ = 0
    total = 0
    for n, m, q, r in _cases(101):
        bc, be, _ = brute.brute_dtw(q, r, f32=True)
        c, e = _double_intermediate_f32(q, r)
        total += 1
        differ += int(not (_same(c, bc) and e == be))
    assert differ >= total // 10, (differ, total)


@pytest.mark.parametrize("f32", [False, True])
def test_enumeration_path_counts(f32):
    """Path counts do not depend on the precision: m(m+1)/2 subsequence
    paths for one event, 1 for one level; Delannoy numbers for global."""
    for m in range(1, 7):
        assert brute.brute_dtw(np.zeros(1, np.float32), np.zeros(m, np.float32), f32=f32)[2] == m * (m + 1) // 2
    delannoy = {(2, 2): 3, (3, 3): 13, (3, 4): 25, (4, 4): 63, (5, 5): 321}
    for (n, m), cnt in delannoy.items():
        assert brute.brute_global_dtw(np.zeros(n, np.float32), np.zeros(m, np.float32), f32=f32)[1] == cnt
