// dtw_band.hip -- banded subsequence DTW (RawAlign, arXiv 2310.05037, Sec.
// 2.4.3): only cells within w levels of the diagonal column c(i) =
// floor(i*m/n) of row i are computed; the others are +inf.  Row -1 is the
// free start (zero), column -1 +inf, and the result is the minimum over the
// band cells of row n-1 (smallest column).
//
// Band-relative lane-striped layout, one wave64 per pair:
//   * the frame of row i is the 64*C columns starting at f(i) = c(i) - w;
//     lane k owns frame positions [kC, kC+C), so the W = 2w+1 band columns
//     sit in positions [0, W) of every row;
//   * the sweep is skewed as in the full-table kernels (lane k computes row
//     t - k at step t); query events and the west neighbour move one lane
//     down per step with DPP wave_shr:1;
//   * chained segments have at least as many events as levels, so the frame
//     moves right by s = c(i) - c(i-1) in {0, 1} per row.  When it moves, a
//     lane's levels and previous-row values shift down by one position; the
//     value entering its last position comes from lane k+1 (its first
//     position, computed earlier in the same step: the lanes run in lockstep)
//     through DPP wave_shl:1, and lane 63's new level from a uniform load
//     issued two steps ahead;
//   * frame positions at or past W are outside the band.  The only one a band
//     cell reads is position W of the previous row (north of position W-1
//     when the frame moves), so that cell is forced to +inf every row.
// Per cell: the two shift selects, v_sub_f32, v_min3_f32 and v_add_f32.
// The device planner (dtw_plan.hip, band mode) writes the sentinels and
// lists the other pairs in two classes by frame width, longest first; each
// class kernel takes its list from a persistent queue, and the two run
// concurrently.
#include "dtw_device.h"

namespace ra {

constexpr int kDppWaveShl1 = 0x130;   // DPP control: whole-wave shift left by one lane

// Lanes 0..62 receive `src` from lane+1; lane 63 keeps `old_v`.
RA_DEV float dpp_shl1(float old_v, float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old_v),
                                                                 __builtin_bit_cast(int, src),
                                                                 kDppWaveShl1, 0xF, 0xF, false));
}

RA_DEV int dpp_shr1_i(int old_v, int src) {
    return __builtin_amdgcn_update_dpp(old_v, src, kDppWaveShr1, 0xF, 0xF, false);
}

// Band state of one pair that every lane shares.
struct BandView {
    const float *q;
    const float *r;
    int n, m, w, W;
};

// Uniform row counter: c = floor(row*m/n) with rem = row*m mod n, advanced
// one row at a time (m <= n: at most one carry per row).
struct RowCounter {
    int c, rem;
};

RA_DEV int advance(RowCounter &rc, int m, int n) {
    rc.rem += m;
    const int carry = rc.rem >= n ? 1 : 0;
    rc.rem -= carry ? n : 0;
    rc.c += carry;
    return carry;
}

// Level at column j >= 0 of the region, read at one uniform address (clamped
// to the last level).  Past the region's end the caller uses +inf instead, at
// the point where it consumes the value, so the load is not waited for here.
RA_DEV float level_raw(__amdgpu_buffer_rsrc_t rs, int j, int m) {
    const int jc = j < m ? j : m - 1;
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, 0, jc * 4, 0));
}

// Forces the previous-row value at frame position W (lane kk, register vk)
// to +inf.  W is odd and C even, so vk is odd (0 means no kill).  Up to 8
// columns per lane, one select per odd register; wider lanes pick the
// register by an indexed move on a vector value (vk is uniform).  A switch
// over vk would be merged into one indexed store and send the arrays to
// scratch memory.
template <int C>
RA_DEV void kill_slot(float (&An)[C], int vk, bool mine) {
    if constexpr (C <= 8) {
#pragma unroll
        for (int v = 1; v < C; v += 2) An[v] = (mine && vk == v) ? kInf : An[v];
    } else {
        typedef float vec_t __attribute__((ext_vector_type(C)));
        vec_t x;
#pragma unroll
        for (int v = 0; v < C; ++v) x[v] = An[v];
        const float cur = x[vk];
        x[vk] = mine ? kInf : cur;
#pragma unroll
        for (int v = 0; v < C; ++v) An[v] = x[v];
    }
}

// One step: row i of this lane (frame shift sh) from Ao to An.
//   qv: the row's event; el: west value of position 0 (row i); ed: the west
//   value of the previous step (row i-1, frame i-1); r63: lane 63's new
//   level when its frame moves; xd: carries lane k+1's first position into
//   lane k (lane 63 holds +inf: past the frame).
template <int C, bool MASKED>
RA_DEV void band_step(bool valid, bool sh, float qv, float el, float ed, float r63, float &xd, int kill_v,
                      bool kill_mine, float (&rv)[C], const float (&Ao)[C], float (&An)[C]) {
    static_assert(C % 2 == 0, "W is odd and C even: position W is never a lane's first position");
    // levels of this row's frame
    const float r0 = sh ? rv[1] : rv[0];
    const float xr = dpp_shl1(r63, r0);
#pragma unroll
    for (int v = 0; v < C - 1; ++v) rv[v] = sh ? rv[v + 1] : rv[v];
    rv[C - 1] = sh ? xr : rv[C - 1];
    // previous row in this row's frame: U(v) = Ao(v + sh); U(-1) from the west
    const float ud = sh ? Ao[0] : ed;
    float up = sh ? Ao[1] : Ao[0];
    float prev = fabsf(qv - rv[0]) + fminf(fminf(ud, up), el);
    xd = dpp_shl1(xd, prev);
    An[0] = (MASKED && !valid) ? Ao[0] : prev;
#pragma unroll
    for (int v = 1; v < C; ++v) {
        const float un = v < C - 1 ? (sh ? Ao[v + 1] : Ao[v]) : (sh ? xd : Ao[C - 1]);
        prev = fabsf(qv - rv[v]) + fminf(fminf(up, un), prev);
        up = un;
        An[v] = (MASKED && !valid) ? Ao[v] : prev;
    }
    kill_slot<C>(An, kill_v, kill_mine);
}

template <int C>
RA_DEV void band_pair(const BandView &bv, float &best, int &bj) {
    const int lane = opaque_lane();
    const int n = bv.n, m = bv.m, w = bv.w, W = bv.W;
    const __amdgpu_buffer_rsrc_t rrs = make_rsrc(bv.r, m);
    const __amdgpu_buffer_rsrc_t qrs = make_rsrc(bv.q, n);
    // Row -1 (all zero: free start) in row 0's frame f(0) = -w.
    float rv[C], A[C], B[C];
#pragma unroll
    for (int v = 0; v < C; ++v) {
        const int j = lane * C + v - w;
        const int jc = j < 0 ? 0 : (j >= m ? m - 1 : j);
        const float lv = bload(rrs, jc);
        rv[v] = (j < 0 || j >= m) ? kInf : lv;
        A[v] = 0.0f;
        B[v] = 0.0f;
    }
    // Position W: register W % C (odd) of lane W / C, if inside the frame.
    const int F = 64 * C;
    const bool has_kill = W < F;
    const int kk = W / C, kv = W % C;
    const int kill_v = has_kill ? kv : 0;   // 0: no register kill
    const bool kill_mine = lane == kk;
    // Uniform counters: lane 0's row t (shift injected at step t) and lane
    // 63's row t - 63 + 2 (its new level, loaded two steps ahead).
    RowCounter c0{0, 0}, c63{0, 0};
    int row63 = -61;   // row of c63
    const int nm1 = n - 1;
    // ela, elb: west value of position 0 at even and odd steps.  elb starts
    // at 0: row -1 (free start) is lane 0's north-west value at row 0.  Lane
    // 0 injects +inf (west of the band); once both registers hold it there,
    // the unmasked steps shift into them in place.  xd likewise keeps +inf
    // in lane 63.
    float qv = 0.0f, ela = 0.0f, elb = 0.0f, xd = kInf;
    int sv = 0;
    float qa = uload(qrs, 0, nm1), qb = uload(qrs, 1, nm1);
    float ra = kInf, rb = kInf;   // lane 63's new levels for steps t, t+1
    bool ra_in = false, rb_in = false;   // ... inside the region (else +inf)
    int sa = 0, sb = 0;           // shifts injected at steps t, t+1 (rows t, t+1)
    // rows 0 and 1: s_0 = 0 (row -1 is in row 0's frame), s_1 = c(1) - c(0)
    sb = n > 1 ? advance(c0, m, n) : 0;
    const int T = (n + 65) & ~1;
    const int ta = T < 64 ? T : 64;
    int tb = n & ~1;
    if (tb < ta) tb = ta;
    int t = 0;
    // Lane 63's look-ahead row and the level entering its frame top f(row) +
    // F - 1 >= w >= 0 when that row's frame moves.  Rows before 1 never move
    // and rows from n on are not computed, so their levels go unused.
    auto next_r63 = [&](bool &in) -> float {
        if (row63 >= 1) advance(c63, m, n);
        ++row63;
        const int j = __builtin_amdgcn_readfirstlane(c63.c - w + F - 1);
        in = j < m;
        return level_raw(rrs, j, m);
    };
#define RA_BAND_STEPS(MASKED)                                                                  \
    {                                                                                         \
        const float q0 = qa, q1 = qb;                                                         \
        const float r0v = ra_in ? ra : kInf, r1v = rb_in ? rb : kInf;                         \
        const int s0 = sa, s1 = sb;                                                           \
        qa = uload(qrs, t + 2, nm1);                                                          \
        qb = uload(qrs, t + 3, nm1);                                                          \
        sa = (t + 2 < n) ? advance(c0, m, n) : 0;                                             \
        sb = (t + 3 < n) ? advance(c0, m, n) : 0;                                             \
        ra = next_r63(ra_in);                                                                 \
        rb = next_r63(rb_in);                                                                 \
        {                                                                                     \
            qv = dpp_shr1(q0, qv);                                                            \
            sv = dpp_shr1_i(s0, sv);                                                          \
            ela = dpp_shr1(MASKED ? kInf : ela, A[C - 1]);                                    \
            const bool valid = !MASKED || (unsigned)(t - lane) < (unsigned)n;                 \
            band_step<C, MASKED>(valid, valid && sv != 0, qv, ela, elb, r0v, xd, kill_v,      \
                                 kill_mine, rv, A, B);                                        \
        }                                                                                     \
        {                                                                                     \
            qv = dpp_shr1(q1, qv);                                                            \
            sv = dpp_shr1_i(s1, sv);                                                          \
            elb = dpp_shr1(MASKED ? kInf : elb, B[C - 1]);                                    \
            const bool valid = !MASKED || (unsigned)(t + 1 - lane) < (unsigned)n;             \
            band_step<C, MASKED>(valid, valid && sv != 0, qv, elb, ela, r1v, xd, kill_v,      \
                                 kill_mine, rv, B, A);                                        \
        }                                                                                     \
    }
    // Fill (t < 64), then steps at which every lane's row is in [0, n)
    // (rows t - 63 >= 1 and t + 1 <= n - 1), then drain.
    for (; t < ta; t += 2) RA_BAND_STEPS(true)
    for (; t < tb; t += 2) RA_BAND_STEPS(false)
    for (; t < T; t += 2) RA_BAND_STEPS(true)
#undef RA_BAND_STEPS
    // Row n-1 in its frame f(n-1) = c(n-1) - w.
    const int f_end = (int)((int64_t)(n - 1) * m / n) - w;
    best = kInf;
    bj = 0x7fffffff;
#pragma unroll
    for (int v = 0; v < C; ++v) {
        const int u = lane * C + v;
        const int j = f_end + u;
        if (u < W && j >= 0 && j < m) take_min(best, bj, A[v], j);
    }
    wave_min(best, bj);
    if (!(best < kInf)) bj = -1;
}

// C = 2H columns per lane for H in [H, HMAX].
template <int H, int HMAX>
RA_DEV void band_dispatch(int h, const BandView &bv, float &best, int &bj) {
    if constexpr (H <= HMAX) {
        if (h == H)
            band_pair<2 * H>(bv, best, bj);
        else
            band_dispatch<H + 1, HMAX>(h, bv, best, bj);
    }
}

// Frames of 128(HLO-1)+1 .. 128 HHI columns.  Every listed pair is valid
// and takes a frame in this range (the planner wrote the others' results).
template <int HLO, int HHI, int WAVES>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WAVES, WAVES)))
void k_band(PairArrays a, const int32_t *__restrict__ band, const int32_t *__restrict__ list,
            const int32_t *__restrict__ count, int32_t *queue) {
    const int n_items = *count;
    int it = 0;
    if (__lane_id() == 0) it = atomicAdd(queue, 1);
    int item = __builtin_amdgcn_readfirstlane(it);
    while (item < n_items) {
        const int p = list[item];
        const int n = a.q_len[p];
        const int m = a.r_len[p];
        const int wraw = band[p];
        // w >= m-1 admits every column of every row: same band
        const int w = wraw < m - 1 ? wraw : m - 1;
        const int W = 2 * w + 1;
        const BandView bv{a.q + a.q_off[p], a.r + a.r_off[p], n, m, w, W};
        const int h = (W + 127) / 128;   // C = 2h columns per lane, 64 C >= W
        float best = __builtin_nanf("");
        int bj = -2;
        band_dispatch<HLO, HHI>(h, bv, best, bj);
        if (__lane_id() == 0) {
            a.out_score[p] = best;
            a.out_end[p] = bj;
        }
        if (__lane_id() == 0) it = atomicAdd(queue, 1);
        item = __builtin_amdgcn_readfirstlane(it);
    }
}

// Class 2: pairs the band-relative frame does not take (more levels than
// events, so the band moves more than one column per row, or a band wider
// than 2048 columns) in regions of at most 2048 levels.  The frame is the
// whole region, as in the full-table kernels (lane k owns columns [kC,
// kC+C)), and every cell outside its row's band is forced to +inf: a
// subtraction, a compare and a select more per cell.  Each lane follows
// c(i) of its own row with a counter.
template <int C>
RA_DEV void band_abs_pair(const BandView &bv, float &best, int &bj) {
    const int lane = opaque_lane();
    const int n = bv.n, m = bv.m, w = bv.w;
    const __amdgpu_buffer_rsrc_t rrs = make_rsrc(bv.r, m);
    const __amdgpu_buffer_rsrc_t qrs = make_rsrc(bv.q, n);
    const int col0 = lane * C;
    float rv[C], A[C];
#pragma unroll
    for (int v = 0; v < C; ++v) {
        const int j = col0 + v;
        const float lv = bload(rrs, j < m ? j : m - 1);
        rv[v] = j < m ? lv : kInf;
        A[v] = 0.0f;   // row -1: the free start
    }
    // c = floor(i*m/n) of this lane's row i, rem = i*m mod n.
    const int qd = m / n, rd = m % n;
    int c = 0, rem = 0;
    // Column -1 is +inf; so is the corner D(-1,-1) here, which gives row 0
    // the same minimum as its north value D(-1,0) = 0.
    float ecur = kInf, eprev, qv = 0.0f;
    const int nm1 = n - 1;
    float qa = uload(qrs, 0, nm1), qb = uload(qrs, 1, nm1);
    const int T = n + 63;
    for (int t = 0; t < T; ++t) {
        const float q0 = qa;
        qa = qb;
        qb = uload(qrs, t + 2, nm1);
        qv = dpp_shr1(q0, qv);
        eprev = ecur;
        ecur = dpp_shr1(kInf, A[C - 1]);
        const int i = t - lane;
        const bool valid = (unsigned)i < (unsigned)n;
        const int a = c - w - col0;   // band of row i in lane positions: [a, a + 2w]
        float diag = eprev, left = ecur;
#pragma unroll
        for (int v = 0; v < C; ++v) {
            const float up = A[v];
            float nv = fabsf(qv - rv[v]) + fminf(fminf(diag, up), left);
            nv = (unsigned)(v - a) <= (unsigned)(2 * w) ? nv : kInf;
            diag = up;
            left = nv;
            A[v] = valid ? nv : A[v];
        }
        if (valid) {
            rem += rd;
            const int carry = rem >= n ? 1 : 0;
            rem -= carry ? n : 0;
            c += qd + carry;
        }
    }
    best = kInf;
    bj = 0x7fffffff;
#pragma unroll
    for (int v = 0; v < C; ++v)
        if (col0 + v < m) take_min(best, bj, A[v], col0 + v);
    wave_min(best, bj);
    if (!(best < kInf)) bj = -1;
}

template <int H>
RA_DEV void band_abs_dispatch(int h, const BandView &bv, float &best, int &bj) {
    if constexpr (H <= kBandMaxFrame / 128) {
        if (h == H)
            band_abs_pair<2 * H>(bv, best, bj);
        else
            band_abs_dispatch<H + 1>(h, bv, best, bj);
    }
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_band_abs(PairArrays a, const int32_t *__restrict__ band, const int32_t *__restrict__ list,
                const int32_t *__restrict__ count, int32_t *queue) {
    const int n_items = *count;
    int it = 0;
    if (__lane_id() == 0) it = atomicAdd(queue, 1);
    int item = __builtin_amdgcn_readfirstlane(it);
    while (item < n_items) {
        const int p = list[item];
        const int n = a.q_len[p];
        const int m = a.r_len[p];
        const int wraw = band[p];
        const int w = wraw < m - 1 ? wraw : m - 1;
        const BandView bv{a.q + a.q_off[p], a.r + a.r_off[p], n, m, w, 2 * w + 1};
        float best = __builtin_nanf("");
        int bj = -2;
        band_abs_dispatch<1>((m + 127) / 128, bv, best, bj);
        if (__lane_id() == 0) {
            a.out_score[p] = best;
            a.out_end[p] = bj;
        }
        if (__lane_id() == 0) it = atomicAdd(queue, 1);
        item = __builtin_amdgcn_readfirstlane(it);
    }
}

// Class 3: regions above 2048 levels that the band-relative frame does not
// take (more levels than events, or a band wider than 2048 columns).  One
// wave sweeps the region stripe by stripe with the multi-stripe kernel's
// shape (S = ceil(m / 2048) stripes of 64 C columns) and, as in class 2,
// forces every cell outside its row's band to +inf.  A stripe over columns
// [a, b] sweeps only the rows whose band meets it: [i0, i1] with i0 the
// first row with c(i) >= a - w and i1 the last with c(i) <= b + w.  Its
// rows before i0 are out of band (+inf; row -1 is the free start, zero),
// and its rows after i1 reach neither row n-1 nor the next stripe, whose
// west column reads +inf outside [i0, i1].  Lane 63 stores the stripe's
// last column of rows [i0, i1] into the wave's edge slot, in place (a row
// is read by a stripe before that stripe rewrites it).
template <int C>
RA_DEV void band_multi_stripe(const BandView &bv, int s, int a, int i0, int i1, int p0, int p1, float *edge,
                              float &best, int &bj) {
    const int lane = opaque_lane();
    const int n = bv.n, m = bv.m, w = bv.w;
    const int col0 = a + lane * C;
    const __amdgpu_buffer_rsrc_t rrs = make_rsrc(bv.r, m);
    const __amdgpu_buffer_rsrc_t qrs = make_rsrc(bv.q, n);
    const __amdgpu_buffer_rsrc_t ers = make_rsrc(edge, n);
    const int nm1 = n - 1;
    float rv[C], A[C];
    const float row_before = i0 == 0 ? 0.0f : kInf;   // row i0 - 1 in this stripe
#pragma unroll
    for (int v = 0; v < C; ++v) {
        const int j = col0 + v;
        const float lv = bload(rrs, j < m ? j : m - 1);
        rv[v] = j < m ? lv : kInf;
        A[v] = row_before;
    }
    // West value of row `row` for lane 0: the previous stripe's last column
    // inside its rows [p0, p1], else +inf (out of band), row -1 zero.
    auto west = [&](int row) -> float {
        const float e = uload(ers, row < 0 ? 0 : row, nm1);
        if (s == 0) return kInf;
        return (row >= p0 && row <= p1) ? e : (row == -1 ? 0.0f : kInf);
    };
    // c(i) = floor(i*m/n) of this lane's row, from row i0 on.
    const int64_t im = (int64_t)i0 * m;
    int c = (int)(im / n), rem = (int)(im % n);
    const int qd = m / n, rd = m % n;
    const int ns = i1 - i0 + 1;
    float ecur = west(i0 - 1), eprev, qv = 0.0f;
    float qa = uload(qrs, i0, nm1), qb = uload(qrs, i0 + 1, nm1);
    float ea = west(i0), eb = west(i0 + 1);
    const int T = ns + 63;
    for (int t = 0; t < T; ++t) {
        const float q0 = qa, e0 = ea;
        qa = qb;
        qb = uload(qrs, i0 + t + 2, nm1);
        ea = eb;
        eb = west(i0 + t + 2);
        qv = dpp_shr1(q0, qv);
        eprev = ecur;
        ecur = dpp_shr1(e0, A[C - 1]);
        const bool valid = (unsigned)(t - lane) < (unsigned)ns;
        const int lo = c - w - col0;   // band of this lane's row in lane positions: [lo, lo + 2w]
        float diag = eprev, left = ecur;
#pragma unroll
        for (int v = 0; v < C; ++v) {
            const float up = A[v];
            float nv = fabsf(qv - rv[v]) + fminf(fminf(diag, up), left);
            nv = (unsigned)(v - lo) <= (unsigned)(2 * w) ? nv : kInf;
            diag = up;
            left = nv;
            A[v] = valid ? nv : A[v];
        }
        if (lane == 63 && valid) edge[i0 + t - 63] = A[C - 1];
        if (valid) {
            rem += rd;
            const int carry = rem >= n ? 1 : 0;
            rem -= carry ? n : 0;
            c += qd + carry;
        }
    }
    best = kInf;
    bj = 0x7fffffff;
    if (i1 == n - 1) {
#pragma unroll
        for (int v = 0; v < C; ++v)
            if (col0 + v < m) take_min(best, bj, A[v], col0 + v);
    }
    wave_min(best, bj);
}

// First row whose diagonal column reaches X, last row whose diagonal column
// is at most Y (c(i) = floor(i*m/n) is non-decreasing).
RA_DEV int first_row_at(int64_t X, int n, int m) { return X <= 0 ? 0 : (int)((X * n + m - 1) / m); }
RA_DEV int last_row_at(int64_t Y, int n, int m) { return Y < 0 ? -1 : (int)(((Y + 1) * n + m - 1) / m) - 1; }

template <int C>
RA_DEV void band_multi_pair(const BandView &bv, int S, float *edge, float &best, int &bj) {
    best = kInf;
    bj = 0x7fffffff;
    int p0 = 1, p1 = 0;   // the previous stripe's rows (none yet)
    for (int s = 0; s < S; ++s) {
        const int a = s * 64 * C;
        const int b = (a + 64 * C < bv.m ? a + 64 * C : bv.m) - 1;
        int i0 = first_row_at((int64_t)a - bv.w, bv.n, bv.m);
        int i1 = last_row_at((int64_t)b + bv.w, bv.n, bv.m);
        i1 = i1 < bv.n - 1 ? i1 : bv.n - 1;
        if (i0 > i1) {   // the band does not meet this stripe
            p0 = 1;
            p1 = 0;
            continue;
        }
        float sb;
        int sj;
        band_multi_stripe<C>(bv, s, a, i0, i1, p0, p1, edge, sb, sj);
        take_min(best, bj, sb, sj);
        p0 = i0;
        p1 = i1;
        // Lane 63's edge stores must be visible to lane 0 of the next stripe.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    if (!(best < kInf)) bj = -1;
}

template <int H>
RA_DEV void band_multi_dispatch(int h, const BandView &bv, int S, float *edge, float &best, int &bj) {
    if constexpr (H <= kMultiMaxH) {
        if (h == H)
            band_multi_pair<kMultiColStep * H>(bv, S, edge, best, bj);
        else
            band_multi_dispatch<H + 1>(h, bv, S, edge, best, bj);
    }
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_band_multi(PairArrays a, const int32_t *__restrict__ band, const int32_t *__restrict__ list,
                  const int32_t *__restrict__ count, int32_t *queue, float *edge_base) {
    float *edge = edge_base + (size_t)blockIdx.x * kEdgeCap;
    const int n_items = *count;
    int it = 0;
    if (__lane_id() == 0) it = atomicAdd(queue, 1);
    int item = __builtin_amdgcn_readfirstlane(it);
    while (item < n_items) {
        const int p = list[item];
        const int n = a.q_len[p];
        const int m = a.r_len[p];
        const int wraw = band[p];
        const int w = wraw < m - 1 ? wraw : m - 1;
        const BandView bv{a.q + a.q_off[p], a.r + a.r_off[p], n, m, w, 2 * w + 1};
        int S, h;
        stripe_shape(m, S, h, false);
        float best = __builtin_nanf("");
        int bj = -2;
        band_multi_dispatch<kMultiMinH>(h, bv, S, edge, best, bj);
        if (__lane_id() == 0) {
            a.out_score[p] = best;
            a.out_end[p] = bj;
        }
        if (__lane_id() == 0) it = atomicAdd(queue, 1);
        item = __builtin_amdgcn_readfirstlane(it);
    }
}

// Class 0 (C <= 8) fits 64 VGPRs: eight waves per SIMD; class 1 four.
#define RA_BAND_LO k_band<1, kBandLoMaxH, 8>
#define RA_BAND_HI k_band<kBandLoMaxH + 1, kBandMaxFrame / 128, 4>

hipError_t launch_band(int cls, const PairArrays &a, const int32_t *band, int grid, const PlanScratch &s,
                       hipStream_t stream) {
    const int32_t *list = s.list + cls * s.capacity;
    const int32_t *count = s.counts + cls;
    int32_t *queue = s.queue + cls;
    if (cls == 0)
        hipLaunchKernelGGL(RA_BAND_LO, dim3((unsigned)grid), dim3(64), 0, stream, a, band, list, count, queue);
    else if (cls == 1)
        hipLaunchKernelGGL(RA_BAND_HI, dim3((unsigned)grid), dim3(64), 0, stream, a, band, list, count, queue);
    else if (cls == 2)
        hipLaunchKernelGGL(k_band_abs, dim3((unsigned)grid), dim3(64), 0, stream, a, band, list, count, queue);
    else   // one edge slot per workgroup: grid <= the slots
        hipLaunchKernelGGL(k_band_multi, dim3((unsigned)grid), dim3(64), 0, stream, a, band, list, count, queue,
                           s.edge);
    return hipGetLastError();
}

int band_blocks_per_cu(int cls) {
    int nb = 0;
    if (cls == 0)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, RA_BAND_LO, 64, 0);
    else if (cls == 1)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, RA_BAND_HI, 64, 0);
    else if (cls == 2)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_band_abs, 64, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_band_multi, 64, 0);
    return nb > 0 ? nb : 1;
}

#undef RA_BAND_LO
#undef RA_BAND_HI

}  // namespace ra
