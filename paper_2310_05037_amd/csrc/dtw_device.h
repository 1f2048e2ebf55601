// dtw_device.h -- device code shared by the gfx950 DTW kernels.
//
// The recurrence (RawAlign, arXiv 2310.05037, Sec. 2.2) is a min-plus
// dynamic program: D(i,j) = |q_i - r_j| + min(D(i-1,j-1), D(i-1,j), D(i,j-1)),
// row -1 all zero (free start in the region), column -1 +inf.  It is not a
// contraction, so it runs on the plain FP32 vector ALUs: one v_sub_f32, one
// v_min3_f32 and one v_add_f32 with an |x| source modifier per cell.
//
// Lane-striped wavefront layout (one wave64 per pair):
//   * the region is cut into S column stripes of 64*C columns; in a stripe
//     lane k owns C consecutive columns and keeps their levels and the
//     current DP row in VGPRs while the wave sweeps every query row;
//   * the sweep is skewed: at step t lane k computes row i = t - k;
//   * the cell left of lane k's first column comes from lane k-1's last
//     column of the previous step, and the query event from lane k-1 as
//     well: both move one lane down per step with a DPP wave_shr:1 move,
//     lane 0 keeping an injected value (bound_ctrl off);
//   * lane 0's injected left value is +inf in the first stripe (column -1)
//     and the previous stripe's last column otherwise; lane 63 writes its
//     last column to a per-wave edge buffer for the next stripe;
//   * the per-lane DP row is double-buffered (A -> B on even steps, B -> A on
//     odd ones), so no register moves are needed inside the loop.
// Fill/drain steps (t < 64 or t > n-1) leave lanes whose row is outside
// [0, n) unchanged through a select; in between all 64 lanes are busy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace ra {

#define RA_DEV __device__ __forceinline__


constexpr float kInf = __builtin_inff();
constexpr int kDppWaveShr1 = 0x138;   // DPP control: whole-wave shift right by one lane
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 buffer descriptor word 3 (32-bit data)

// Lanes 1..63 receive `src` from lane-1; lane 0 keeps `old_v`.
RA_DEV float dpp_shr1(float old_v, float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old_v),
                                                                 __builtin_bit_cast(int, src),
                                                                 kDppWaveShr1, 0xF, 0xF, false));
}

// One DP cell: rounded subtraction, exact |.|, exact min of three, rounded add.
RA_DEV float cell(float qv, float rv, float diag, float up, float left) {
    const float d = qv - rv;
    return fabsf(d) + fminf(fminf(diag, up), left);
}

// One query row over the lane's C columns.  Ao = previous row of this lane,
// diag/left = the previous and current row's value in the column left of the
// lane, An = new row.
template <int C>
RA_DEV void row_step(const float (&rv)[C], float qv, float diag, float left, const float (&Ao)[C],
                     float (&An)[C]) {
    An[0] = cell(qv, rv[0], diag, Ao[0], left);
#pragma unroll
    for (int s = 1; s < C; ++s) An[s] = cell(qv, rv[s], Ao[s - 1], Ao[s], An[s - 1]);
}

// Fill/drain form: lanes whose row is outside [0, n) copy the previous row
// instead (a select, not a branch, so the old and new rows never have to be
// live at the same time).  Once a lane is past its last row both buffers
// hold that row.
template <int C>
RA_DEV void row_step_masked(bool valid, const float (&rv)[C], float qv, float diag, float left,
                            const float (&Ao)[C], float (&An)[C]) {
    float prev = cell(qv, rv[0], diag, Ao[0], left);
    An[0] = valid ? prev : Ao[0];
#pragma unroll
    for (int s = 1; s < C; ++s) {
        prev = cell(qv, rv[s], Ao[s - 1], Ao[s], prev);
        An[s] = valid ? prev : Ao[s];
    }
}

// Two-chain form (lane skew 2): the first half of the lane's columns
// [0, H) computes row i while the second half [H, C) computes row i-1, so
// every step carries two independent min-plus chains.  Ao holds [row i-1 |
// row i-2] and An receives [row i | row i-1]; An[H-1] still holds row i-2
// of the first half on entry, which is the second half's north-west
// neighbour, so it is read before the first chain overwrites it.  v1/v2:
// the rows of the two halves lie in [0, n) (only read when MASKED).
template <int C, bool MASKED>
RA_DEV void row_step2(bool v1, bool v2, const float (&rv)[C], float q1, float q2, float diag, float left,
                      const float (&Ao)[C], float (&An)[C]) {
    constexpr int H = C / 2;
    const float d2 = An[H - 1];
    float f = cell(q1, rv[0], diag, Ao[0], left);
    float g = cell(q2, rv[H], d2, Ao[H], Ao[H - 1]);
    An[0] = (MASKED && !v1) ? Ao[0] : f;
    An[H] = (MASKED && !v2) ? Ao[H] : g;
#pragma unroll
    for (int s = 1; s < H; ++s) {
        f = cell(q1, rv[s], Ao[s - 1], Ao[s], f);
        g = cell(q2, rv[H + s], Ao[H + s - 1], Ao[H + s], g);
        An[s] = (MASKED && !v1) ? Ao[s] : f;
        An[H + s] = (MASKED && !v2) ? Ao[H + s] : g;
    }
}

// Buffer resource over n floats at p.  Every caller passes one pair's (or one
// stripe's) pointer, the same in every lane of the wave; reading it from the
// first lane tells the compiler so, which keeps the resource in scalar
// registers.  Otherwise each buffer load in a sweep is wrapped in a loop
// over the distinct resources of the active lanes.
RA_DEV __amdgpu_buffer_rsrc_t make_rsrc(const float *p, int n) {
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
    const int bytes = __builtin_amdgcn_readfirstlane(n * 4);
    float *base = reinterpret_cast<float *>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, bytes, kRsrcWord3);
}

// Element t (clamped to [0, nm1]) of a buffer, read at one uniform address by
// every lane; only lane 0 keeps it after the DPP shift.  rev: element nm1 - t
// instead (query read back to front).
RA_DEV float uload(__amdgpu_buffer_rsrc_t rs, int t, int nm1, bool rev = false) {
    const int tt = t < nm1 ? t : nm1;
    const int ix = rev ? nm1 - tt : tt;
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, 0, ix * 4, 0));
}

RA_DEV float bload(__amdgpu_buffer_rsrc_t rs, int idx) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, idx * 4, 0, 0));
}

// Lane id, opaque to the optimiser.  Every column count has its own code
// path inside a persistent loop over pairs; if the lane-derived values of all
// paths were hoisted out of that loop they would stay live together and
// exhaust the register file.
RA_DEV int opaque_lane() {
    int lane = __lane_id();
    asm volatile("" : "+v"(lane));
    return lane;
}

// Lexicographic (value, column) minimum: smallest value, then smallest column.
RA_DEV void take_min(float &best, int &bj, float v, int j) {
    if (v < best || (v == best && j < bj)) {
        best = v;
        bj = j;
    }
}

RA_DEV void wave_min(float &best, int &bj) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float ov = __shfl_xor(best, off, 64);
        const int oj = __shfl_xor(bj, off, 64);
        take_min(best, bj, ov, oj);
    }
}

struct PairView {
    const float *q;
    int n;
    const float *r;
    int m;
    float *row;   // resident row (streaming) or null
    bool fresh;              // row -1 is the boundary (not a resident row)
    bool corner = false;     // boundary: only the corner D(-1,-1) = 0, the rest of row -1 +inf
    bool fixed_end = false;  // result: D(n-1, m-1) instead of the minimum of row n-1
    bool reverse = false;    // query and region read back to front
};

template <bool EXT>
RA_DEV PairView pair_view(const PairArrays &a, int p) {
    PairView pv;
    pv.q = a.q + a.q_off[p];
    pv.n = a.q_len[p];
    pv.r = a.r + a.r_off[p];
    pv.m = a.r_len[p];
    pv.row = EXT ? a.rows + a.row_off[p] : nullptr;
    pv.fresh = EXT ? a.first_chunk[p] != 0 : true;
    pv.corner = !EXT && a.bound != kBoundSubseq;
    pv.fixed_end = !EXT && a.bound == kBoundGlobal;
    pv.reverse = !EXT && a.reverse != 0;
    return pv;
}

// Slices inside q and r (and the resident row), lengths within the limits
// of the striped kernels.
RA_DEV bool slices_ok(const PairArrays &a, int64_t p, bool extend) {
    const int n = a.q_len[p];
    const int m = a.r_len[p];
    const int64_t qo = a.q_off[p];
    const int64_t ro = a.r_off[p];
    bool ok = n >= 0 && m >= 0 && qo >= 0 && ro >= 0 && qo + n <= a.q_size && ro + m <= a.r_size &&
              m <= kMaxRegion && n <= kMaxQuery && (m <= kSingleMaxRegion || n <= kEdgeCap);
    if (extend) {
        const int64_t wo = a.row_off[p];
        ok = ok && wo >= 0 && wo + m <= a.rows_size;
    }
    return ok;
}

// A valid global pair narrow enough for one lane (dtw_global.hip).
RA_DEV bool tiny_pair(const PairArrays &a, int64_t p) {
    const int n = a.q_len[p];
    const int m = a.r_len[p];
    return a.bound == kBoundGlobal && !a.reverse && n >= 1 && m >= 1 && m <= kTinyMaxCols &&
           slices_ok(a, p, false);
}

// Registers of one lane: levels, the double-buffered DP row.  Columns are
// tested against lim = m - col0 (one register) rather than by their index,
// so no per-column index stays live through the sweep.  Row -1 is zero for
// a fresh subsequence alignment, +inf for the corner boundary (its corner
// D(-1,-1) = 0 enters through lane 0's north-west value instead).  Reversed
// pairs read column j from r[m-1-j].
template <int C, bool EXT>
RA_DEV void load_lane(const PairView &pv, int col0, float (&rv)[C], float (&A)[C], float (&B)[C]) {
    const int lim = pv.m - col0;
    const int last = lim - 1;
    const __amdgpu_buffer_rsrc_t rrs = make_rsrc(pv.r, pv.m);
    __amdgpu_buffer_rsrc_t wrs = rrs;
    if (EXT) wrs = make_rsrc(pv.row, pv.m);
    const float row0 = pv.corner ? kInf : 0.0f;
#pragma unroll
    for (int s = 0; s < C; ++s) {
        const int jc = col0 + (s < last ? s : last);   // clamped into the region
        const float lv = bload(rrs, pv.reverse ? pv.m - 1 - jc : jc);
        rv[s] = s < lim ? lv : 0.0f;   // padding columns: finite, never reported
        float init = row0;
        if (EXT && !pv.fresh) {
            const float iv = bload(wrs, jc);
            init = s < lim ? iv : 0.0f;
        }
        A[s] = init;
        B[s] = init;
    }
}

// After the sweep every lane has had at least one step past its last row,
// so A holds row n-1 (or row -1 when n == 0).  Reduce it and optionally
// store it.  A global alignment reports column m-1 only.
template <int C, bool EXT>
RA_DEV void finish_lane(const PairView &pv, int col0, const float (&A)[C], float &best, int &bj) {
    const int lim = pv.m - col0;
    best = kInf;
    bj = 0x7fffffff;
    if (!EXT && pv.fixed_end) {
#pragma unroll
        for (int s = 0; s < C; ++s)
            if (s == lim - 1) take_min(best, bj, A[s], col0 + s);
        return;
    }
#pragma unroll
    for (int s = 0; s < C; ++s) {
        if (s < lim) {
            take_min(best, bj, A[s], col0 + s);
            if (EXT) pv.row[col0 + s] = A[s];
        }
    }
}

// Two consecutive steps (t even: A -> B, t+1: B -> A).  EIN: lane 0's left
// values e0/e1 come from the edge buffer.  Else lane 0's E0 stays +inf
// (column -1) and its E1 is refilled from E0, so E1's initial value (the
// corner D(-1,-1), 0 for a global alignment) is used once, as row 0's
// north-west value.  EOUT: lane 63 writes its last column of the rows it
// finished to edge[].
template <int C, bool MASKED, bool EIN, bool EOUT>
RA_DEV void two_steps(int t, int n, int lane, const float (&rv)[C], float (&A)[C], float (&B)[C],
                      float &qv, float q0, float q1, float &E0, float &E1, float e0, float e1,
                      float *edge) {
    qv = dpp_shr1(q0, qv);
    E0 = dpp_shr1(EIN ? e0 : E0, A[C - 1]);
    if (MASKED) row_step_masked<C>((unsigned)(t - lane) < (unsigned)n, rv, qv, E1, E0, A, B);
    else row_step<C>(rv, qv, E1, E0, A, B);
    if (EOUT && t >= 63 && t - 63 < n && lane == 63) edge[t - 63] = B[C - 1];
    qv = dpp_shr1(q1, qv);
    E1 = dpp_shr1(EIN ? e1 : E0, B[C - 1]);   // lane 0 without an edge: column -1, +inf
    if (MASKED) row_step_masked<C>((unsigned)(t + 1 - lane) < (unsigned)n, rv, qv, E0, E1, B, A);
    else row_step<C>(rv, qv, E0, E1, B, A);
    if (EOUT && t >= 62 && t - 62 < n && lane == 63) edge[t - 62] = A[C - 1];
}

// Two-chain version of two_steps (see row_step2): lane k computes row
// t - 2k in its first half and row t - 2k - 1 in its second half.  Qe/Qo
// hold the first half's query event of the even/odd steps; the second
// half's event is the other register.  Lane 63's second half finishes row
// t - 127 at step t.
template <int C, bool MASKED, bool EIN, bool EOUT>
RA_DEV void two_steps2(int t, int n, int lane, const float (&rv)[C], float (&A)[C], float (&B)[C],
                       float &Qe, float &Qo, float q0, float q1, float &E0, float &E1, float e0, float e1,
                       float *edge) {
    Qe = dpp_shr1(q0, Qe);
    E0 = dpp_shr1(EIN ? e0 : E0, A[C - 1]);
    row_step2<C, MASKED>((unsigned)(t - 2 * lane) < (unsigned)n, (unsigned)(t - 2 * lane - 1) < (unsigned)n,
                         rv, Qe, Qo, E1, E0, A, B);
    if (EOUT && t >= 127 && t - 127 < n && lane == 63) edge[t - 127] = B[C - 1];
    Qo = dpp_shr1(q1, Qo);
    E1 = dpp_shr1(EIN ? e1 : E0, B[C - 1]);
    row_step2<C, MASKED>((unsigned)(t + 1 - 2 * lane) < (unsigned)n, (unsigned)(t - 2 * lane) < (unsigned)n,
                         rv, Qo, Qe, E0, E1, B, A);
    if (EOUT && t >= 126 && t - 126 < n && lane == 63) edge[t - 126] = A[C - 1];
}

// Cross-wave hand-over hook of the sweep (the multi-wave pipeline,
// dtw_pipe.hip).  NoSync, the default, is compiled out entirely.  An active
// policy is called every kBlock steps of the sweep:
//   wait(rows):     before the edge values of rows < rows are loaded (the
//                   stripe to the left must have stored them); false after a
//                   time-out, and the sweep then runs on without waiting;
//   publish(rows):  after this stripe's lane 63 has stored the edge values of
//                   rows < rows;
//   set_corner(v):  this stripe's row -1 value in its last column, handed
//                   to the next stripe before any row is published;
//   corner():       the corner left of this stripe, read after the first wait.
struct NoSync {
    static constexpr bool kActive = false;
    static constexpr int kBlock = 64;
    RA_DEV bool wait(int) { return true; }
    RA_DEV void publish(int) {}
    RA_DEV void set_corner(float) {}
    RA_DEV float corner() { return 0.0f; }
};

// One column stripe [col_base, col_base + 64*C) of a pair on one wave.
// Returns this stripe's (min, argmin) of row n-1 over columns < m.  ILP2:
// two independent chains per lane and step (lane skew 2, see row_step2),
// which pays off on long queries; else one chain (lane skew 1).
//   corner:      D(-1, col_base-1), row -1 left of this stripe (read when EIN);
//   next_corner: receives D(-1, col_base+64C-1) for the next stripe.  Both
//                travel in registers because the resident row is updated in
//                place, stripe by stripe.
template <int C, bool EXT, bool EIN, bool EOUT, bool ILP2, class SYNC = NoSync>
RA_DEV void sweep(const PairView &pv, int col_base, float *edge, float corner, float &next_corner, float &best,
                  int &bj, SYNC *sync = nullptr) {
    static_assert(!SYNC::kActive || !ILP2, "the hand-over assumes a skew of one lane per step");
    const int lane = opaque_lane();
    const int col0 = col_base + lane * C;
    float rv[C], A[C], B[C];
    load_lane<C, EXT>(pv, col0, rv, A, B);
    next_corner = __shfl(A[C - 1], 63, 64);
    if constexpr (SYNC::kActive) {
        if (EOUT) sync->set_corner(next_corner);
    }
    const int n = pv.n;
    if (n > 0) {
        // Left boundary of the region: D(i,-1) = +inf for every row.  At row
        // 0 the corner D(-1,-1) of a subsequence alignment may be 0, but then
        // D(-1,0) = 0 as well, so +inf gives the same minimum; a global
        // alignment enters through that corner, which is 0.
        float E0 = kInf, E1 = pv.corner ? 0.0f : kInf, qv = 0.0f, qo = 0.0f;
        if (EIN) E1 = corner;   // row 0's north-west neighbour left of this stripe
        const __amdgpu_buffer_rsrc_t qrs = make_rsrc(pv.q, n);
        const __amdgpu_buffer_rsrc_t ers = make_rsrc(edge, n);
        const int nm1 = n - 1;
        // Every lane gets at least one step past its last row.
        const int skew = ILP2 ? 128 : 64;    // steps until lane 63 starts its last rows
        const int T = (n + skew + 1) & ~1;      // >= n + skew steps, even
        const int ta = T < skew ? T : skew;     // end of the masked fill
        int tb = n & ~1;                        // end of the unmasked middle
        if (tb < ta) tb = ta;
        const bool qrev = pv.reverse;
        float qa = uload(qrs, 0, nm1, qrev), qb = uload(qrs, 1, nm1, qrev);
        float ea = 0.0f, eb = 0.0f;
        if (EIN) {
            if constexpr (SYNC::kActive) {
                // rows [0, kBlock + 2) before the first loads; the corner
                // was handed over before any row was published
                (void)sync->wait(n < SYNC::kBlock + 2 ? n : SYNC::kBlock + 2);
                E1 = sync->corner();
            }
            ea = uload(ers, 0, nm1);
            eb = uload(ers, 1, nm1);
        }
        int t = 0;
        // Every kBlock steps: wait for the edge rows the next kBlock steps
        // load (up to t + kBlock + 1) and publish the rows lane 63 has
        // stored (it stores row u - 63 at step u, so steps 0 .. t-1 stored
        // rows 0 .. t-64).
#define RA_SYNC_POINT                                                                        \
    if constexpr (SYNC::kActive) {                                                           \
        if ((t & (SYNC::kBlock - 1)) == 0) {                                                 \
            if (EIN) {                                                                       \
                const int need = t + SYNC::kBlock + 2;                                       \
                (void)sync->wait(need < n ? need : n);                                       \
            }                                                                                \
            if (EOUT) {                                                                      \
                const int done = t - 63;                                                     \
                sync->publish(done < 0 ? 0 : (done < n ? done : n));                         \
            }                                                                                \
        }                                                                                    \
    }
#define RA_STEPS(MASKED)                                                                     \
    {                                                                                        \
        RA_SYNC_POINT                                                                        \
        const float q0 = qa, q1 = qb, e0 = ea, e1 = eb;                                      \
        qa = uload(qrs, t + 2, nm1, qrev);                                                   \
        qb = uload(qrs, t + 3, nm1, qrev);                                                   \
        if (EIN) {                                                                           \
            ea = uload(ers, t + 2, nm1);                                                     \
            eb = uload(ers, t + 3, nm1);                                                     \
        }                                                                                    \
        if constexpr (ILP2)                                                                  \
            two_steps2<C, MASKED, EIN, EOUT>(t, n, lane, rv, A, B, qv, qo, q0, q1, E0, E1, e0, e1, edge); \
        else                                                                                 \
            two_steps<C, MASKED, EIN, EOUT>(t, n, lane, rv, A, B, qv, q0, q1, E0, E1, e0, e1, edge); \
    }
        for (; t < ta; t += 2) RA_STEPS(true)
        for (; t < tb; t += 2) RA_STEPS(false)
        for (; t < T; t += 2) RA_STEPS(true)
#undef RA_STEPS
#undef RA_SYNC_POINT
        if constexpr (SYNC::kActive) {
            if (EOUT) sync->publish(n);   // every edge row is stored
        }
    }
    finish_lane<C, EXT>(pv, col0, A, best, bj);
    wave_min(best, bj);
}

// Stripe shape of a region of m levels: S stripes of 64*C columns,
// C = step h.  single: the pair is on a single-stripe route (one stripe,
// the smallest h with 64 C >= m, step kSingleColStep).  Otherwise S =
// ceil(m / (256 kMultiMaxK)) and the smallest h with S * 64 C >= m, step
// kMultiColStep; then every stripe starts inside the region ((S-1)*64*C < m
// over the whole range of m).  Returns the padded columns of one stripe, 64 C.
RA_DEV int stripe_shape(int m, int &S, int &h, bool single) {
    const int width = single ? kSingleMaxRegion : 256 * kMultiMaxK;
    const int group = 64 * (single ? kSingleColStep : kMultiColStep);
    S = (m + width - 1) / width;
    if (S < 1) S = 1;
    h = (m + group * S - 1) / (group * S);
    return group * h;
}

// Narrowest and widest multi-stripe lanes: the smallest h over every region
// that can take the multi-stripe route (above the lowest single-stripe
// cut-off, 2048 levels, up to kMaxRegion), and 4 kMultiMaxK / step.
constexpr int multi_min_h() {
    int hmin = 4 * kMultiMaxK / kMultiColStep;
    for (int m = kSingleLoMaxRegion + 1; m <= kMaxRegion; ++m) {
        const int w = 256 * kMultiMaxK;
        const int S = (m + w - 1) / w;
        const int h = (m + 64 * kMultiColStep * S - 1) / (64 * kMultiColStep * S);
        if (h < hmin) hmin = h;
    }
    return hmin;
}
constexpr int kMultiMinH = multi_min_h();
constexpr int kMultiMaxH = 4 * kMultiMaxK / kMultiColStep;

// Two independent min-plus chains per lane (the lane's two column halves one
// row apart); the skew per stripe grows from 64 to 128 steps.  Off by
// default: at four waves per SIMD the other waves supply the independent
// work and the shorter skew wins.
#ifndef RA_MULTI_ILP2
#define RA_MULTI_ILP2 0
#endif
constexpr bool kMultiIlp2 = RA_MULTI_ILP2 != 0;
static_assert(!kMultiIlp2 || kMultiColStep == 2, "the two-chain sweep needs an even column count");

// One pair swept stripe by stripe by one wave (several stripes when the
// region is wider than one): lane 63 stores each stripe's last column into
// the wave's edge slot, lane 0 of the next stripe reads it back.  Returns
// the minimum of the pair's last row and its smallest column.
template <int C, bool EXT>
RA_DEV void multi_pair(const PairView &pv, int S, float *edge, float &best, int &bj) {
    best = kInf;
    bj = 0x7fffffff;
    float corner = 0.0f;   // D(-1, col_base-1) of the next stripe
    for (int s = 0; s < S; ++s) {
        float b, nc;
        int j;
        if (s == 0)
            sweep<C, EXT, false, true, kMultiIlp2>(pv, 0, edge, 0.0f, nc, b, j);
        else
            sweep<C, EXT, true, true, kMultiIlp2>(pv, s * 64 * C, edge, corner, nc, b, j);
        corner = nc;
        take_min(best, bj, b, j);
        // Lane 63's edge stores must be visible to lane 0 of the next stripe.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

}  // namespace ra
