"""Host-side pin of the two-lanes-per-gap schedule of the anchored gap kernel.

A global DTW gap (Sec. 2.4.2: entered from the corner D(-1,-1) = 0, the rest
of row -1 and column -1 at +inf, cost D(n-1, m-1)) of a width class W sits
right-aligned in W slots, the pad W - m slots on the left holding +inf
levels.  In the classes W = 24 .. 64 two lanes share a gap: the first holds
slots [0, W/2), the second slots [W/2, W) and runs one row behind, taking
the west value of its first slot from the first lane's last slot of that
row (handed over once per row) and its north-west value from the row
before.  Neither lane peels off a step: the second lane's first step works
on a row before the gap, which must leave its row -1 at +inf.  That holds
because every region of these classes is wider than W/2 (the class below
is at least half as wide), so the corner slot pad - 1 lies in the first
half.

Modelled here step by step in float32 and compared bit for bit with the
plain table, on random gaps of every paired class, the widest and narrowest
regions of each, and queries of one event upward.  Independent of the
oracle and of the kernel.
"""
import numpy as np

INF = np.float32(np.inf)
WIDTHS = [4, 8, 12, 16, 24, 32, 48, 64]   # width classes; the last four are paired


def _cell(q, r, diag, up, left):
    return np.float32(np.float32(abs(np.float32(q - r))) + min(min(diag, up), left))


def _plain(q, r):
    """Global DTW table in float32, row by row; returns D(n-1, m-1)."""
    m = len(r)
    prev = [INF] * m
    corner = np.float32(0)
    for qi in q:
        cur = [INF] * m
        for j in range(m):
            diag = (corner if j == 0 else prev[j - 1])
            left = INF if j == 0 else cur[j - 1]
            cur[j] = _cell(qi, r[j], diag, prev[j], left)
        corner = INF
        prev = cur
    return prev[m - 1]


def _two_lanes(q, r, W):
    """The paired schedule: per step the first lane computes row s, the
    second row s - 1; the result is the second lane's last slot at row n-1."""
    H, n, m = W // 2, len(q), len(r)
    pad = W - m
    lanes = []
    for half in (0, 1):
        v0 = half * H
        lanes.append({
            "rv": [np.float32(r[v0 + v - pad]) if v0 + v >= pad else INF for v in range(H)],
            "row": [np.float32(0) if v0 + v == pad - 1 else INF for v in range(H)],
            "corner": np.float32(0) if half == 0 and pad == 0 else INF,
            "last": INF, "edge_prev": INF,
        })
    res = None
    for s in range(n + 1):
        lasts = (lanes[0]["last"], lanes[1]["last"])   # handed over between steps
        for half in (0, 1):
            L = lanes[half]
            qv = q[min(max(s - half, 0), n - 1)]
            edge = lasts[1 - half]
            nw0 = L["edge_prev"] if half else L["corner"]
            w0 = edge if half else INF
            old, new = L["row"], [None] * H
            new[0] = _cell(qv, L["rv"][0], nw0, old[0], w0)
            for v in range(1, H):
                new[v] = _cell(qv, L["rv"][v], old[v - 1], old[v], new[v - 1])
            L["corner"], L["edge_prev"], L["last"], L["row"] = INF, edge, new[H - 1], new
            if half and s == n:
                res = new[H - 1]
    return res


def test_paired_classes_keep_the_corner_in_the_first_half():
    for c in range(4, len(WIDTHS)):
        W, below = WIDTHS[c], WIDTHS[c - 1]
        assert W - (below + 1) < W // 2      # largest pad of the class


def test_two_lane_schedule_equals_the_table():
    rng = np.random.default_rng(11)
    checked = 0
    for c in range(4, len(WIDTHS)):
        W, below = WIDTHS[c], WIDTHS[c - 1]
        shapes = [(1, below + 1), (1, W), (2, W), (3, below + 1)]
        shapes += [(int(rng.integers(1, 30)), int(rng.integers(below + 1, W + 1))) for _ in range(30)]
        for n, m in shapes:
            q = rng.standard_normal(n).astype(np.float32)
            r = rng.standard_normal(m).astype(np.float32)
            if rng.random() < 0.3:   # small integers: many equal neighbours
                q = rng.integers(0, 3, n).astype(np.float32)
                r = rng.integers(0, 3, m).astype(np.float32)
            got, exp = _two_lanes(q, r, W), _plain(q, r)
            assert np.float32(got).view(np.uint32) == np.float32(exp).view(np.uint32), (W, n, m, got, exp)
            checked += 1
    assert checked == 4 * 34
