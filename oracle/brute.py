"""Brute-force subsequence DTW by enumerating every warping path.

TEST INFRASTRUCTURE ONLY (tiny inputs).  Independent of the recurrence in
dtw_oracle.c: instead of a table it walks every path explicitly.

A path (RawAlign Sec. 2.2: each step comes from the north, north-west or west
neighbour) is a sequence of cells that starts in row 0 at any column, moves by
(1,0), (0,1) or (1,1), and stops at any cell of row n-1.  Its cost is the sum
of |q_i - r_j| over its cells, accumulated in path order (double precision
unless f32=True).
The subsequence DTW cost is the smallest path cost; the end is the smallest
final column among the cheapest paths.

Because a rounded addition is monotone (x <= y implies fl(x + c) <= fl(y + c)),
the table recurrence returns exactly the smallest rounded path sum, so this
enumeration matches it bit for bit on any input, not only on exactly
representable ones.  That holds in either precision, as long as the path sum
rounds like the table does.  With f32=True every cost is |fl32(q_i - r_j)|
and every running sum is rounded to float32 after each cell (numpy float32
scalars), which pins the oracle's float instantiations on ordinary inputs:
a float recurrence that keeps any intermediate in double, or takes the
difference in double, disagrees with it.
"""
from __future__ import annotations

import math
import sys

import numpy as np


def _cost_table(q, r, f32: bool):
    """c[i][j] = |q_i - r_j| as Python floats (double: the difference of the
    float inputs widened to double) or numpy float32 scalars (float: the
    difference rounded to float32, then its magnitude), and the zero of the
    running sums in the same type."""
    if f32:
        qf = np.asarray(q, dtype=np.float32)
        rf = np.asarray(r, dtype=np.float32)
        return [[np.float32(abs(qf[i] - rf[j])) for j in range(len(rf))] for i in range(len(qf))], np.float32(0)
    qd = [float(x) for x in q]
    rd = [float(x) for x in r]
    return [[abs(qd[i] - rd[j]) for j in range(len(rd))] for i in range(len(qd))], 0.0


def enumerate_paths(n: int, m: int):
    """Yield every path as a list of (i, j) cells (small n, m only)."""
    path = []

    def walk(i, j):
        path.append((i, j))
        if i == n - 1:
            yield list(path)
        if i + 1 < n:
            yield from walk(i + 1, j)
        if j + 1 < m:
            yield from walk(i, j + 1)
        if i + 1 < n and j + 1 < m:
            yield from walk(i + 1, j + 1)
        path.pop()

    for j0 in range(m):
        yield from walk(0, j0)


def brute_dtw(q, r, f32: bool = False):
    """(cost, end, number of paths) by explicit path enumeration.  f32: the
    costs and running sums are float32 (see the module note)."""
    n, m = len(q), len(r)
    if n == 0:
        return 0.0, -1, 0
    if m == 0:
        return math.inf, -1, 0
    c, _ = _cost_table(q, r, f32)
    sys.setrecursionlimit(max(1000, 4 * (n + m) + 100))
    best = math.inf
    best_end = -1
    count = 0
    # Depth-first walk with the running sum, so paths are not materialised.
    stack = [(0, j0, c[0][j0]) for j0 in reversed(range(m))]
    while stack:
        i, j, acc = stack.pop()
        if i == n - 1:
            count += 1
            if acc < best or (acc == best and j < best_end):
                best, best_end = acc, j
        if i + 1 < n:
            stack.append((i + 1, j, acc + c[i + 1][j]))
        if j + 1 < m:
            stack.append((i, j + 1, acc + c[i][j + 1]))
        if i + 1 < n and j + 1 < m:
            stack.append((i + 1, j + 1, acc + c[i + 1][j + 1]))
    return best, best_end, count


def brute_global_dtw(q, r, f32: bool = False):
    """(cost, number of paths) of global DTW between two anchors by explicit
    enumeration: every path starts at cell (0, 0), moves by (1,0), (0,1) or
    (1,1) and stops at (n-1, m-1) (Sec. 2.4.2: the gap is entered and left
    through the anchor corners).  Empty on both sides: (0, 1); empty on one
    side only: (+inf, 0).  f32: float32 costs and running sums."""
    n, m = len(q), len(r)
    if n == 0 or m == 0:
        return (0.0, 1) if n == 0 and m == 0 else (math.inf, 0)
    c, _ = _cost_table(q, r, f32)
    best = math.inf
    count = 0
    stack = [(0, 0, c[0][0])]
    while stack:
        i, j, acc = stack.pop()
        if i == n - 1 and j == m - 1:
            count += 1
            best = min(best, acc)
            continue
        if i + 1 < n:
            stack.append((i + 1, j, acc + c[i + 1][j]))
        if j + 1 < m:
            stack.append((i, j + 1, acc + c[i][j + 1]))
        if i + 1 < n and j + 1 < m:
            stack.append((i + 1, j + 1, acc + c[i + 1][j + 1]))
    return best, count


def brute_span(q, r, f32: bool = False):
    """(cost, end, start) by explicit enumeration of subsequence paths (as
    brute_dtw): the cheapest cost, the smallest final column among the
    cheapest paths, and among the cheapest paths ending there the largest
    first column.  Empty query: (0, -1, -1); empty region: (+inf, -1, -1).

    f32: cost and end as brute_dtw(f32=True).  The start is then defined by
    sums taken backwards, as the alignment is re-read from its end: every
    path from (n-1, end) back to row 0 is summed in float32 from its last
    cell to its first, and the start is the largest first column among the
    paths with the smallest such sum.  In exact arithmetic both directions
    give the same set of optimal paths; in float the backward sums decide."""
    n, m = len(q), len(r)
    if n == 0:
        return 0.0, -1, -1
    if m == 0:
        return math.inf, -1, -1
    c, _ = _cost_table(q, r, f32)
    if f32:
        cost, end, _ = brute_dtw(q, r, f32=True)
        # Walk backwards from the end cell: north, west, north-west; every
        # cell of row 0 reached is a possible first cell.
        bsum, bstart = math.inf, -1
        stack = [(n - 1, end, c[n - 1][end])]
        while stack:
            i, j, acc = stack.pop()
            if i == 0 and (acc < bsum or (acc == bsum and j > bstart)):
                bsum, bstart = acc, j
            if i > 0:
                stack.append((i - 1, j, acc + c[i - 1][j]))
            if j > 0:
                stack.append((i, j - 1, acc + c[i][j - 1]))
            if i > 0 and j > 0:
                stack.append((i - 1, j - 1, acc + c[i - 1][j - 1]))
        return cost, end, bstart
    best = {}   # end column -> (cost, largest start among that cost)
    stack = [(0, j0, j0, c[0][j0]) for j0 in range(m)]
    while stack:
        i, j, s0, acc = stack.pop()
        if i == n - 1:
            cc, st = best.get(j, (math.inf, -1))
            if acc < cc or (acc == cc and s0 > st):
                best[j] = (acc, s0)
        if i + 1 < n:
            stack.append((i + 1, j, s0, acc + c[i + 1][j]))
        if j + 1 < m:
            stack.append((i, j + 1, s0, acc + c[i][j + 1]))
        if i + 1 < n and j + 1 < m:
            stack.append((i + 1, j + 1, s0, acc + c[i + 1][j + 1]))
    cost = min(cc for cc, _ in best.values())
    end = min(j for j, (cc, _) in best.items() if cc == cost)
    return cost, end, best[end][1]


def brute_band(q, r, w, f32: bool = False):
    """(cost, end) of banded subsequence DTW by enumeration: every
    subsequence path (as brute_dtw) whose cells all satisfy
    |j - floor(i*m/n)| <= w; the cheapest cost, the smallest final column.
    No path: (+inf, -1).  f32: float32 costs and running sums."""
    n, m = len(q), len(r)
    if n == 0:
        return 0.0, -1
    if m == 0:
        return math.inf, -1
    c, _ = _cost_table(q, r, f32)

    def ok(i, j):
        return abs(j - (i * m) // n) <= w

    best, best_end = math.inf, -1
    stack = [(0, j0, c[0][j0]) for j0 in range(m) if ok(0, j0)]
    while stack:
        i, j, acc = stack.pop()
        if i == n - 1:
            if acc < best or (acc == best and j < best_end):
                best, best_end = acc, j
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            i2, j2 = i + di, j + dj
            if i2 < n and j2 < m and ok(i2, j2):
                stack.append((i2, j2, acc + c[i2][j2]))
    return best, best_end


def brute_path(q, r, start, end):
    """The warping path that the tie rule of the path oracle selects, by
    explicit enumeration: among all paths from (0, start) to (n-1, end)
    whose cost (summed in double, path order) is the smallest, the one whose
    moves read backwards from (n-1, end) are first in the order north-west <
    north < west.  Returns (cost, lo, hi) with lo[i] .. hi[i] the columns of
    row i.  Use exactly representable inputs, so that equal costs are equal
    in double."""
    q = [float(x) for x in q]
    r = [float(x) for x in r]
    n = len(q)
    best = None
    # Paths walked backwards from (n-1, end): each step is NW (0), N (1), W (2).
    stack = [((n - 1, end), abs(q[n - 1] - r[end]), ())]
    while stack:
        (i, j), acc, moves = stack.pop()
        if i == 0 and j == start:
            key = (acc, moves)
            if best is None or key < best:
                best = key
            continue
        if i > 0 and j > start:
            stack.append(((i - 1, j - 1), acc + abs(q[i - 1] - r[j - 1]), moves + (0,)))
        if i > 0:
            stack.append(((i - 1, j), acc + abs(q[i - 1] - r[j]), moves + (1,)))
        if j > start:
            stack.append(((i, j - 1), acc + abs(q[i] - r[j - 1]), moves + (2,)))
    cost, moves = best
    lo = [0] * n
    hi = [0] * n
    i, j = n - 1, end
    hi[i] = j
    lo[i] = j
    for mv in moves:
        if mv == 2:
            j -= 1
        else:
            if mv == 0:
                j -= 1
            i -= 1
            hi[i] = j
        lo[i] = j
    return cost, lo, hi


def brute_path_f32(q, r, start, end):
    """The float warping path by enumeration, for ordinary (not exactly
    summable) inputs.  For every cell (i, j) of the interval [start, end],
    P(i, j) is the smallest float32 sum, taken in path order, over every path
    from (0, start) to (i, j) (all of them are enumerated).  The path is then
    read back from (n-1, end): at each cell the next one is the neighbour
    with the smallest P among north-west, north and west (inside the
    interval), the first of them in that order on ties.  In float two paths
    through different neighbours can round to the same sum, so the choice
    is made on the neighbours' sums, not on the whole path's.
    Returns (cost P(n-1, end), lo, hi)."""
    n = len(q)
    L = end - start + 1
    c, _ = _cost_table(q, r[start:end + 1], True)
    P = [[math.inf] * L for _ in range(n)]
    stack = [(0, 0, c[0][0])]
    while stack:
        i, j, acc = stack.pop()
        if acc < P[i][j]:
            P[i][j] = acc
        if i + 1 < n:
            stack.append((i + 1, j, acc + c[i + 1][j]))
        if j + 1 < L:
            stack.append((i, j + 1, acc + c[i][j + 1]))
        if i + 1 < n and j + 1 < L:
            stack.append((i + 1, j + 1, acc + c[i + 1][j + 1]))
    lo = [0] * n
    hi = [0] * n
    i, j = n - 1, L - 1
    hi[i] = lo[i] = start + j
    while (i, j) != (0, 0):
        moves = []
        if i > 0 and j > 0:
            moves.append((P[i - 1][j - 1], 0, i - 1, j - 1))
        if i > 0:
            moves.append((P[i - 1][j], 1, i - 1, j))
        if j > 0:
            moves.append((P[i][j - 1], 2, i, j - 1))
        _, _, i2, j2 = min(moves)
        if i2 != i:
            hi[i2] = start + j2
        i, j = i2, j2
        lo[i] = start + j
    return P[n - 1][L - 1], lo, hi
