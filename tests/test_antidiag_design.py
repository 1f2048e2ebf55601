"""Host-side pin of the row reduction the anti-diagonal kernel relies on.

Below query row n-1 the kernel's thread t_l computes its remaining rows with
a weight of 0 on the distance term, D(i, j) = min(D(i-1, j-1), D(i-1, j),
D(i, j-1)), with column -1 at +inf, and reads the minimum and its first
column from its last row instead of row n-1.  Such a row is the prefix
minimum of the row above, so the minimum and the first column holding it
are those of row n-1 (min is exact in float32; Sec. 2.4.4 takes the
subsequence score as the minimum of the last row, smallest column on ties).
Brute force here on small float32 tables with many ties, independent of the
oracle and of the kernel.
"""
import numpy as np

INF = np.float32(np.inf)


def _table(q, r, weights):
    """Rows of the subsequence DTW table in float32, row i's distance term
    scaled by weights[i] (1 or 0), row -1 = 0, column -1 = +inf."""
    prev = np.zeros(len(r), np.float32)
    rows = []
    for qi, c in zip(q, weights):
        cur = np.empty(len(r), np.float32)
        w, nw = INF, (np.float32(0) if not rows else INF)
        for j, rj in enumerate(r):
            cost = np.float32(abs(np.float32(qi - rj))) if c else np.float32(0)
            cur[j] = np.float32(cost + min(nw, prev[j], w))
            nw, w = prev[j], cur[j]
        rows.append(cur)
        prev = cur
    return rows


def test_weight_zero_rows_keep_minimum_and_first_column():
    rng = np.random.default_rng(2)
    checked = 0
    for _ in range(400):
        n, m, pad = int(rng.integers(1, 7)), int(rng.integers(1, 24)), int(rng.integers(1, 8))
        if rng.random() < 0.5:
            q = rng.integers(0, 3, n + pad).astype(np.float32)   # small integers: many equal sums
            r = rng.integers(0, 3, m).astype(np.float32)
        else:
            q = rng.standard_normal(n + pad).astype(np.float32)
            r = rng.standard_normal(m).astype(np.float32)
        rows = _table(q, r, [1] * n + [0] * pad)
        last, below = rows[n - 1], rows[-1]
        assert below[-1] == last.min()                       # prefix minimum ends at the row minimum
        assert np.all(np.diff(below) <= 0)                   # non-increasing
        assert below.min() == last.min() and int(np.argmin(below)) == int(np.argmin(last))
        checked += 1
    assert checked == 400


def test_weight_zero_row_is_prefix_minimum():
    rng = np.random.default_rng(3)
    for _ in range(100):
        m = int(rng.integers(1, 40))
        q = rng.integers(0, 4, 3).astype(np.float32)
        r = rng.integers(0, 4, m).astype(np.float32)
        rows = _table(q, r, [1, 1, 0])
        assert np.array_equal(rows[2], np.minimum.accumulate(rows[1]))
