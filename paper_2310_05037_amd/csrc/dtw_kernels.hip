// dtw_kernels.hip -- gfx950 kernels for batched subsequence DTW.
//
// The recurrence (RawAlign, arXiv 2310.05037, Sec. 2.2) is a min-plus
// dynamic program: D(i,j) = |q_i - r_j| + min(D(i-1,j-1), D(i-1,j), D(i,j-1)),
// row -1 all zero (free start in the region), column -1 +inf.  It is not a
// contraction, so it runs on the plain FP32 vector ALUs: one v_sub_f32, one
// v_min3_f32 and one v_add_f32 with an |x| source modifier per cell.
//
// Lane-striped wavefront layout (one wave64 per pair, or per column stripe):
//   * lane k owns C consecutive region columns [kC, kC+C) and keeps their
//     levels r and the current DP row in VGPRs for the whole query;
//   * the wave sweeps query rows in a skewed schedule: at step t lane k
//     computes row i = t - k, so each step every lane updates C cells;
//   * the cell left of lane k's first column comes from lane k-1's last
//     column of the previous step, and the query event from lane k-1 as
//     well: both move one lane down per step with a DPP wave_shr:1 move,
//     lane 0 keeping the injected value (bound_ctrl off);
//   * the per-lane DP row is double-buffered (A -> B on even steps, B -> A on
//     odd ones) so no register moves are needed inside the loop.
// Fill/drain steps (t < 64 or t > n-1) mask lanes whose row is outside
// [0, n); in between all 64 lanes are busy.
//
// Long regions use several waves of one workgroup, each wave owning a
// column stripe of 64*C columns.  Wave w hands its last column to wave w+1
// through a ring buffer in LDS; waves advance in blocks of kBlock steps
// separated by workgroup barriers, wave w lagging wave w-1 by kLag blocks.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "rawalign.h"

namespace ra {

#define RA_DEV __device__ __forceinline__

constexpr float kInf = __builtin_inff();
constexpr int kDppWaveShr1 = 0x138;          // DPP control: whole-wave shift right by one lane
constexpr int kRsrcWord3 = 0x00020000;       // gfx9 buffer descriptor word 3 (32-bit data)
constexpr int kBlock = 32;                   // steps between barriers (cooperative kernels)
constexpr int kLag = 3;                      // blocks between consecutive waves (>= 1 + 62/kBlock)
constexpr int kRing = 256;                   // LDS ring entries per wave boundary
constexpr int kRingMask = kRing - 1;
constexpr int kMaxQuery = 1 << 28;              // keeps 4*n and the step counter in int

static_assert(kLag * kBlock >= kBlock + 63, "a wave must see its left neighbour's edge a block early");

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

RA_DEV float qload(__amdgpu_buffer_rsrc_t rs, int t, int nm1) {
    // Uniform address (clamped in scalar registers): every lane reads q[t];
    // only lane 0 keeps it after the DPP shift.
    const int tt = t < nm1 ? t : nm1;
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, 0, tt * 4, 0));
}

RA_DEV __amdgpu_buffer_rsrc_t make_rsrc(const float *p, int n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), (short)0, n * 4, kRsrcWord3);
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
    bool fresh;   // row -1 is all zero
};

// Lane id, opaque to the optimiser.  Every column count has its own code
// path inside a persistent loop over pairs; if the lane-derived values of all
// paths were hoisted out of that loop they would stay live together and
// exhaust the register file.
RA_DEV int opaque_lane() {
    int lane = __lane_id();
    asm volatile("" : "+v"(lane));
    return lane;
}

RA_DEV float bload(__amdgpu_buffer_rsrc_t rs, int idx) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, idx * 4, 0, 0));
}

// Registers of one lane: levels, the double-buffered DP row.  Columns are
// tested against lim = m - col0 (one register) rather than by their index,
// so no per-column index stays live through the sweep.
template <int C, bool EXT>
RA_DEV void load_lane(const PairView &pv, int col0, float (&rv)[C], float (&A)[C], float (&B)[C]) {
    const int lim = pv.m - col0;
    const int last = lim - 1;
    const __amdgpu_buffer_rsrc_t rrs = make_rsrc(pv.r, pv.m);
    __amdgpu_buffer_rsrc_t wrs = rrs;
    if (EXT) wrs = make_rsrc(pv.row, pv.m);
#pragma unroll
    for (int s = 0; s < C; ++s) {
        const int jc = col0 + (s < last ? s : last);   // clamped into the region
        const float lv = bload(rrs, jc);
        rv[s] = s < lim ? lv : 0.0f;   // padding columns: finite, never reported
        float init = 0.0f;
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
// store it.
template <int C, bool EXT>
RA_DEV void finish_lane(const PairView &pv, int col0, const float (&A)[C], float &best, int &bj) {
    const int lim = pv.m - col0;
    best = kInf;
    bj = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < C; ++s) {
        if (s < lim) {
            take_min(best, bj, A[s], col0 + s);
            if (EXT) pv.row[col0 + s] = A[s];
        }
    }
}

// Two consecutive steps (t even: A -> B, t+1: B -> A) of a single-wave sweep.
template <int C, bool MASKED>
RA_DEV void two_steps(int t, int n, int lane, const float (&rv)[C], float (&A)[C], float (&B)[C],
                      float &qv, float q0, float q1, float &E0, float &E1) {
    qv = dpp_shr1(q0, qv);
    E0 = dpp_shr1(E0, A[C - 1]);
    if (MASKED) row_step_masked<C>((unsigned)(t - lane) < (unsigned)n, rv, qv, E1, E0, A, B);
    else row_step<C>(rv, qv, E1, E0, A, B);
    qv = dpp_shr1(q1, qv);
    E1 = dpp_shr1(E1, B[C - 1]);
    if (MASKED) row_step_masked<C>((unsigned)(t + 1 - lane) < (unsigned)n, rv, qv, E0, E1, B, A);
    else row_step<C>(rv, qv, E0, E1, B, A);
}

// One pair on one wave: region columns [0, 64*C) cover m.
template <int C, bool EXT>
RA_DEV void wave_pair(const PairView &pv, float &best, int &bj) {
    const int lane = opaque_lane();
    const int col0 = lane * C;
    float rv[C], A[C], B[C];
    load_lane<C, EXT>(pv, col0, rv, A, B);
    const int n = pv.n;
    if (n > 0) {
        // Left boundary: D(i,-1) = +inf for every row.  At row 0 the corner
        // D(-1,-1) may be 0, but then D(-1,0) = 0 as well, so +inf gives the
        // same minimum.
        float E0 = kInf, E1 = kInf, qv = 0.0f;
        const __amdgpu_buffer_rsrc_t qrs = make_rsrc(pv.q, n);
        const int nm1 = n - 1;
        const int T = (n + 65) & ~1;            // >= n + 64 steps, even
        const int ta = T < 64 ? T : 64;        // end of the masked fill
        int tb = n & ~1;                        // end of the unmasked middle
        if (tb < ta) tb = ta;
        float qa = qload(qrs, 0, nm1), qb = qload(qrs, 1, nm1);
        int t = 0;
        for (; t < ta; t += 2) {
            const float q0 = qa, q1 = qb;
            qa = qload(qrs, t + 2, nm1);
            qb = qload(qrs, t + 3, nm1);
            two_steps<C, true>(t, n, lane, rv, A, B, qv, q0, q1, E0, E1);
        }
        for (; t < tb; t += 2) {
            const float q0 = qa, q1 = qb;
            qa = qload(qrs, t + 2, nm1);
            qb = qload(qrs, t + 3, nm1);
            two_steps<C, false>(t, n, lane, rv, A, B, qv, q0, q1, E0, E1);
        }
        for (; t < T; t += 2) {
            const float q0 = qa, q1 = qb;
            qa = qload(qrs, t + 2, nm1);
            qb = qload(qrs, t + 3, nm1);
            two_steps<C, true>(t, n, lane, rv, A, B, qv, q0, q1, E0, E1);
        }
    }
    finish_lane<C, EXT>(pv, col0, A, best, bj);
    wave_min(best, bj);
}

// ---- cooperative (multi-wave) sweep for long regions -----------------------

template <int C, bool MASKED>
RA_DEV void two_steps_ring(int t, int n, int lane, const float (&rv)[C], float (&A)[C],
                           float (&B)[C], float &qv, float q0, float q1, float &E0, float &E1,
                           const float *ring_in, float *ring_out) {
    qv = dpp_shr1(q0, qv);
    E0 = dpp_shr1(ring_in[t & kRingMask], A[C - 1]);
    if (MASKED) row_step_masked<C>((unsigned)(t - lane) < (unsigned)n, rv, qv, E1, E0, A, B);
    else row_step<C>(rv, qv, E1, E0, A, B);
    if (lane == 63 && t >= 63) ring_out[(t - 63) & kRingMask] = B[C - 1];
    qv = dpp_shr1(q1, qv);
    E1 = dpp_shr1(ring_in[(t + 1) & kRingMask], B[C - 1]);
    if (MASKED) row_step_masked<C>((unsigned)(t + 1 - lane) < (unsigned)n, rv, qv, E0, E1, B, A);
    else row_step<C>(rv, qv, E0, E1, B, A);
    if (lane == 63 && t >= 62) ring_out[(t - 62) & kRingMask] = A[C - 1];
}

// One pair on the W waves of a workgroup.  ring: (W+1)*kRing floats in LDS;
// ring[0..kRing) holds +inf (left boundary of wave 0), wave w reads ring
// w and writes ring w+1.  red_v/red_j: W entries each.
template <int C, bool EXT>
RA_DEV void coop_pair(const PairView &pv, int W, int wave, float *ring, float *red_v, int *red_j,
                      float &best, int &bj) {
    const int lane = opaque_lane();
    const int col0 = (wave * 64 + lane) * C;
    float rv[C], A[C], B[C];
    load_lane<C, EXT>(pv, col0, rv, A, B);
    const int n = pv.n;
    if (n > 0) {
        float E0 = kInf, E1 = kInf, qv = 0.0f;
        if (wave > 0) {
            // Row 0's north-west neighbour left of this stripe: D(-1, col0-1).
            float d0 = 0.0f;
            if (EXT && !pv.fresh) {
                const int jj = wave * 64 * C - 1;
                d0 = jj < pv.m ? pv.row[jj] : 0.0f;
            }
            E1 = d0;
        }
        const float *ring_in = ring + wave * kRing;
        float *ring_out = ring + (wave + 1) * kRing;
        const __amdgpu_buffer_rsrc_t qrs = make_rsrc(pv.q, n);
        const int nm1 = n - 1;
        const int nblk = (n + 64 + kBlock - 1) / kBlock;   // kBlock*nblk >= n + 64 steps
        const int G = nblk + kLag * (W - 1);
        float qa = qload(qrs, 0, nm1), qb = qload(qrs, 1, nm1);
        for (int g = 0; g < G; ++g) {
            const int lb = g - kLag * wave;
            if (lb >= 0 && lb < nblk) {
                const int t0 = lb * kBlock;
                for (int t = t0; t < t0 + kBlock; t += 2) {
                    const float q0 = qa, q1 = qb;
                    qa = qload(qrs, t + 2, nm1);
                    qb = qload(qrs, t + 3, nm1);
                    if (t >= 64 && t + 1 <= nm1)
                        two_steps_ring<C, false>(t, n, lane, rv, A, B, qv, q0, q1, E0, E1, ring_in, ring_out);
                    else
                        two_steps_ring<C, true>(t, n, lane, rv, A, B, qv, q0, q1, E0, E1, ring_in, ring_out);
                }
            }
            __syncthreads();
        }
    }
    float wb;
    int wj;
    finish_lane<C, EXT>(pv, col0, A, wb, wj);
    wave_min(wb, wj);
    if (lane == 0) {
        red_v[wave] = wb;
        red_j[wave] = wj;
    }
    __syncthreads();
    best = red_v[0];
    bj = red_j[0];
    for (int w = 1; w < W; ++w) take_min(best, bj, red_v[w], red_j[w]);
    __syncthreads();   // red_* and the rings are reused by the next pair
}

// ---- work distribution -----------------------------------------------------

template <bool EXT>
RA_DEV PairView pair_view(const PairArrays &a, int p) {
    PairView pv;
    pv.q = a.q + a.q_off[p];
    pv.n = a.q_len[p];
    pv.r = a.r + a.r_off[p];
    pv.m = a.r_len[p];
    pv.row = EXT ? a.rows + a.row_off[p] : nullptr;
    pv.fresh = EXT ? a.first_chunk[p] != 0 : true;
    return pv;
}

RA_DEV void write_result(const PairArrays &a, int p, float best, int bj) {
    a.out_score[p] = best;
    a.out_end[p] = bj;
}

// Short pairs: one wave per pair.  Columns per lane C = 4k, k = ceil(m/256),
// for k in [KLO, KHI] (two kernels: the small-C one runs at higher occupancy).
template <bool EXT, int KLO, int KHI>
RA_DEV void short_dispatch(const PairView &pv, float &best, int &bj) {
    const int k = (pv.m + 255) >> 8;
    best = __builtin_nanf("");
    bj = -2;
#define RA_CASE(K) \
    if (K >= KLO && K <= KHI && k == K) wave_pair<4 * K, EXT>(pv, best, bj);
    RA_CASE(1) RA_CASE(2) RA_CASE(3) RA_CASE(4) RA_CASE(5) RA_CASE(6) RA_CASE(7) RA_CASE(8)
    RA_CASE(9) RA_CASE(10) RA_CASE(11) RA_CASE(12) RA_CASE(13) RA_CASE(14) RA_CASE(15) RA_CASE(16)
#undef RA_CASE
}

// Occupancy targets: at most 32 columns per lane fit 128 VGPRs (4 waves per
// SIMD), up to 64 columns fit 256 (2 waves per SIMD).
template <bool EXT, int KLO, int KHI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KHI <= 8 ? 4 : 2, KHI <= 8 ? 4 : 2))) void k_short(PairArrays a, const int32_t *__restrict__ list,
                                              const int32_t *__restrict__ count, int32_t *queue) {
    const int n_items = *count;
    int item = blockIdx.x;
    if (queue) {
        int it = 0;
        if (__lane_id() == 0) it = atomicAdd(queue, 1);
        item = __builtin_amdgcn_readfirstlane(it);
    }
    while (item < n_items) {
        const int p = list[item];
        const PairView pv = pair_view<EXT>(a, p);
        float best;
        int bj;
        short_dispatch<EXT, KLO, KHI>(pv, best, bj);
        if (__lane_id() == 0) write_result(a, p, best, bj);
        if (!queue) break;
        int it = 0;
        if (__lane_id() == 0) it = atomicAdd(queue, 1);
        item = __builtin_amdgcn_readfirstlane(it);
    }
}

// Long pairs: W = blockDim.x / 64 waves per pair, C = 4k, k = ceil(m / (256 W)).
template <bool EXT>
RA_DEV void coop_dispatch(const PairView &pv, int W, int wave, float *ring, float *red_v, int *red_j,
                          float &best, int &bj) {
    const int k = (pv.m + 256 * W - 1) / (256 * W);
    best = __builtin_nanf("");
    bj = -2;
#define RA_CASE(K) \
    if (k == K) coop_pair<4 * K, EXT>(pv, W, wave, ring, red_v, red_j, best, bj);
    RA_CASE(1) RA_CASE(2) RA_CASE(3) RA_CASE(4) RA_CASE(5) RA_CASE(6) RA_CASE(7) RA_CASE(8)
    RA_CASE(9) RA_CASE(10) RA_CASE(11) RA_CASE(12) RA_CASE(13) RA_CASE(14) RA_CASE(15) RA_CASE(16)
#undef RA_CASE
}

template <bool EXT>
__global__ __launch_bounds__(512) void k_long(PairArrays a, const int32_t *__restrict__ list,
                                              const int32_t *__restrict__ count, int32_t *queue) {
    __shared__ float ring[(kMaxCoopWaves + 1) * kRing];
    __shared__ float red_v[kMaxCoopWaves];
    __shared__ int red_j[kMaxCoopWaves];
    __shared__ int item_s;
    const int W = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int i = threadIdx.x; i < kRing; i += blockDim.x) ring[i] = kInf;
    const int n_items = *count;
    bool first = true;
    for (;;) {
        if (threadIdx.x == 0) {
            if (queue) item_s = atomicAdd(queue, 1);
            else item_s = first ? (int)blockIdx.x : n_items;
        }
        first = false;
        __syncthreads();
        const int item = item_s;
        if (item >= n_items) break;
        const int p = list[item];
        const PairView pv = pair_view<EXT>(a, p);
        float best;
        int bj;
        coop_dispatch<EXT>(pv, W, wave, ring, red_v, red_j, best, bj);
        if (threadIdx.x == 0) write_result(a, p, best, bj);
    }
}

// ---- planning ----------------------------------------------------------------

struct PlanArgs {
    PairArrays a;
    int64_t n_pairs;
    int short_max;
    int coop_waves;
    int buckets;      // 1: single bucket (plain), kBuckets: LPT buckets
    int extend;
    PlanScratch s;
};

// Route of pair p.  Returns -1 when the pair needs no kernel; then
// (*score, *end) is its result: a sentinel for invalid slices (NaN, -2) or
// the value of a degenerate pair (empty query or empty region).
RA_DEV int classify(const PlanArgs &pa, int64_t p, int &bucket, float &score, int &end) {
    const PairArrays &a = pa.a;
    const int n = a.q_len[p];
    const int m = a.r_len[p];
    const int64_t qo = a.q_off[p];
    const int64_t ro = a.r_off[p];
    bool ok = n >= 0 && m >= 0 && qo >= 0 && ro >= 0 && qo + n <= a.q_size && ro + m <= a.r_size &&
              m <= kMaxRegion && n <= kMaxQuery;
    bool fresh = true;
    if (pa.extend) {
        const int64_t wo = a.row_off[p];
        ok = ok && wo >= 0 && wo + m <= a.rows_size;
        fresh = a.first_chunk[p] != 0;
    }
    if (!ok) {
        score = __builtin_nanf("");
        end = -2;
        return -1;
    }
    if (n == 0 && fresh) {
        score = 0.0f;
        end = -1;
        return -1;
    }
    if (m == 0) {
        score = n == 0 ? 0.0f : kInf;
        end = -1;
        return -1;
    }
    int route;
    if (m <= pa.short_max) route = m <= kShortLoMaxRegion ? kRouteShortLo : kRouteShortHi;
    else route = m <= kShortMaxRegion * pa.coop_waves ? kRouteLong : kRouteHuge;
    bucket = 0;
    if (pa.buckets > 1) {
        // Longest-processing-time order: quarter-octave buckets of n*m,
        // bucket 0 holding the largest pairs.
        const float cells = (float)n * (float)m + 1.0f;
        int b = (int)(4.0f * __log2f(cells));
        b = b < 0 ? 0 : (b >= pa.buckets ? pa.buckets - 1 : b);
        bucket = pa.buckets - 1 - b;
    }
    return route;
}

__global__ void k_plan_zero(PlanScratch s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNumRoutes * kBuckets) s.hist[i] = 0;
    if (i < kNumRoutes) {
        s.counts[i] = 0;
        s.queue[i] = 0;
    }
}

__global__ void k_plan_count(PlanArgs pa) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= pa.n_pairs) return;
    int b = 0, e = 0;
    float sc = 0.0f;
    const int route = classify(pa, p, b, sc, e);
    if (route >= 0) {
        atomicAdd(&pa.s.hist[route * kBuckets + b], 1);
    } else {
        pa.a.out_score[p] = sc;
        pa.a.out_end[p] = e;
    }
}

// Exclusive scan of each route's histogram (bucket 0 first) -> cursors.
__global__ void k_plan_scan(PlanScratch s) {
    const int route = threadIdx.x;
    if (route >= kNumRoutes) return;
    int run = 0;
    for (int b = 0; b < kBuckets; ++b) {
        const int c = s.hist[route * kBuckets + b];
        s.hist[route * kBuckets + b] = run;
        run += c;
    }
    s.counts[route] = run;
    s.queue[route] = 0;
}

__global__ void k_plan_scatter(PlanArgs pa) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= pa.n_pairs) return;
    int b = 0, e = 0;
    float sc = 0.0f;
    const int route = classify(pa, p, b, sc, e);
    if (route < 0) return;
    const int pos = atomicAdd(&pa.s.hist[route * kBuckets + b], 1);
    pa.s.list[route * pa.s.capacity + pos] = (int32_t)p;
}

// ---- mapping decision (Sec. 2.3) ----------------------------------------------

__global__ void k_decide(const float *__restrict__ score, int64_t n_pairs, const int64_t *__restrict__ cand_off,
                         const int32_t *__restrict__ cand_cnt, const int32_t *__restrict__ n_events,
                         int64_t n_reads, double b_match, double threshold, int32_t *out_best,
                         double *out_score, uint8_t *out_mapped) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_reads) return;
    const int64_t p0 = cand_off[k];
    const int cnt = cand_cnt[k];
    if (cnt < 0 || p0 < 0 || p0 + cnt > n_pairs) {   // candidate range outside the score array
        out_best[k] = -2;
        out_score[k] = __builtin_nan("");
        out_mapped[k] = 0;
        return;
    }
    const double bonus = b_match * (double)n_events[k];
    int32_t best = -1;
    double bs = -__builtin_inf();
    for (int c = 0; c < cnt; ++c) {
        const double s = bonus - (double)score[p0 + c];
        if (best < 0 || s > bs) {
            best = (int32_t)(p0 + c);
            bs = s;
        }
    }
    out_best[k] = best;
    out_score[k] = bs;
    out_mapped[k] = (best >= 0 && bs >= threshold) ? 1 : 0;
}

// ---- host launchers -------------------------------------------------------------

static PlanArgs plan_args(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s) {
    PlanArgs pa;
    pa.a = a;
    pa.n_pairs = n_pairs;
    pa.short_max = cfg.short_max;
    pa.coop_waves = cfg.coop_waves;
    pa.buckets = cfg.persistent ? kBuckets : 1;
    pa.extend = a.rows != nullptr;
    pa.s = s;
    return pa;
}

hipError_t launch_plan(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                       hipStream_t stream) {
    const PlanArgs pa = plan_args(a, n_pairs, cfg, s);
    hipLaunchKernelGGL(k_plan_zero, dim3((kNumRoutes * kBuckets + 255) / 256), dim3(256), 0, stream, s);
    const unsigned g = (unsigned)((n_pairs + 255) / 256);
    hipLaunchKernelGGL(k_plan_count, dim3(g), dim3(256), 0, stream, pa);
    hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(64), 0, stream, s);
    hipLaunchKernelGGL(k_plan_scatter, dim3(g), dim3(256), 0, stream, pa);
    return hipGetLastError();
}

template <int KLO, int KHI>
static hipError_t launch_short_route(int route, int pgrid, const PairArrays &a, int64_t n_pairs,
                                     const LaunchCfg &cfg, const PlanScratch &s, hipStream_t stream) {
    const int32_t *list = s.list + route * s.capacity;
    const int32_t *count = s.counts + route;
    int32_t *queue = cfg.persistent ? s.queue + route : nullptr;
    const unsigned grid = cfg.persistent ? (unsigned)pgrid : (unsigned)n_pairs;
    if (a.rows)
        hipLaunchKernelGGL((k_short<true, KLO, KHI>), dim3(grid), dim3(64), 0, stream, a, list, count, queue);
    else
        hipLaunchKernelGGL((k_short<false, KLO, KHI>), dim3(grid), dim3(64), 0, stream, a, list, count, queue);
    return hipGetLastError();
}

hipError_t launch_short_lo(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                           hipStream_t stream) {
    return launch_short_route<1, 8>(kRouteShortLo, cfg.short_lo_grid, a, n_pairs, cfg, s, stream);
}

hipError_t launch_short_hi(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                           hipStream_t stream) {
    return launch_short_route<9, 16>(kRouteShortHi, cfg.short_hi_grid, a, n_pairs, cfg, s, stream);
}

static hipError_t launch_coop(int route, int waves, int pgrid, const PairArrays &a, int64_t n_pairs,
                              const LaunchCfg &cfg, const PlanScratch &s, hipStream_t stream) {
    const int32_t *list = s.list + route * s.capacity;
    const int32_t *count = s.counts + route;
    int32_t *queue = cfg.persistent ? s.queue + route : nullptr;
    const unsigned grid = cfg.persistent ? (unsigned)pgrid : (unsigned)n_pairs;
    if (a.rows)
        hipLaunchKernelGGL(k_long<true>, dim3(grid), dim3(64 * waves), 0, stream, a, list, count, queue);
    else
        hipLaunchKernelGGL(k_long<false>, dim3(grid), dim3(64 * waves), 0, stream, a, list, count, queue);
    return hipGetLastError();
}

hipError_t launch_long(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                       hipStream_t stream) {
    return launch_coop(kRouteLong, cfg.coop_waves, cfg.long_grid, a, n_pairs, cfg, s, stream);
}

hipError_t launch_huge(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                       hipStream_t stream) {
    return launch_coop(kRouteHuge, kMaxCoopWaves, cfg.huge_grid, a, n_pairs, cfg, s, stream);
}

hipError_t launch_decide(const float *score, int64_t n_pairs, const int64_t *cand_off, const int32_t *cand_cnt,
                         const int32_t *n_events, int64_t n_reads, double b_match, double threshold,
                         int32_t *out_best, double *out_score, uint8_t *out_mapped, hipStream_t stream) {
    const unsigned g = (unsigned)((n_reads + 255) / 256);
    hipLaunchKernelGGL(k_decide, dim3(g), dim3(256), 0, stream, score, n_pairs, cand_off, cand_cnt, n_events, n_reads,
                       b_match, threshold, out_best, out_score, out_mapped);
    return hipGetLastError();
}

int short_blocks_per_cu(bool extend, bool hi) {
    int nb = 0;
    if (extend && hi)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_short<true, 9, 16>, 64, 0);
    else if (extend)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_short<true, 1, 8>, 64, 0);
    else if (hi)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_short<false, 9, 16>, 64, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_short<false, 1, 8>, 64, 0);
    return nb > 0 ? nb : 1;
}

int long_blocks_per_cu(int coop_waves, bool extend, bool antidiag) {
    (void)antidiag;
    int nb = 0;
    if (extend)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_long<true>, 64 * coop_waves, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_long<false>, 64 * coop_waves, 0);
    return nb > 0 ? nb : 1;
}

}  // namespace ra
