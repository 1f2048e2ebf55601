// dtw_global.hip -- anchor-guided alignment (RawAlign, arXiv 2310.05037,
// Sec. 2.4.2): global DTW of the gaps between consecutive anchors of a chain,
// and the sums of a chain's gap costs.
//
// A gap is entered diagonally from the upper-left anchor and left diagonally
// into the lower-right one: D(-1,-1) = 0, the rest of row -1 and column -1
// are +inf, and the gap costs D(n-1, m-1).  Gaps are short (tens of events
// against a few to a few dozen levels), far too narrow for a 64-lane stripe,
// so here one lane aligns one gap:
//   * the gap's levels and a double-buffered DP row sit in the lane's VGPRs,
//     right-aligned in W slots (W = 4 .. 64), so the result D(n-1, m-1) is
//     always slot W-1;
//   * the W-m slots on the left hold +inf levels: their cells stay +inf and
//     act as column -1; row -1 is +inf except the corner D(-1,-1) = 0 in
//     slot W-m-1 (or left of slot 0 when m == W);
//   * every cell is one v_sub_f32, one v_min3_f32 and one v_add_f32 with an
//     |x| modifier, with no cross-lane traffic at all;
//   * the lanes of a wave take gaps of one width class with similar query
//     lengths (planned on the device: width class, then quarter octaves of
//     n, longest first), so little of a wave idles;
//   * the four widest classes (W = 24 .. 64) take two lanes per gap, one
//     per half of the slots, the second a row behind (k_tiny_pair).
// Gaps wider than 64 levels go to the striped kernels in global mode.
#include "dtw_device.h"

namespace ra {

constexpr int kTinyBins = kTinyClasses * kTinyBuckets;   // 1024
constexpr int kTinyPlanBlock = 1024;   // a few pairs per thread, as in the main planner

RA_DEV int tiny_class(int m) {
    int c = 0;
    while (c < kTinyClasses - 1 && tiny_width(c) < m) ++c;
    return c;
}

// Width class, then query length in quarter octaves, longest first.
RA_DEV int tiny_bin(int n, int m) {
    int b = (int)(4.0f * __log2f((float)n));
    b = b < 0 ? 0 : (b >= kTinyBuckets ? kTinyBuckets - 1 : b);
    return tiny_class(m) * kTinyBuckets + (kTinyBuckets - 1 - b);
}

__global__ void k_tiny_zero(TinyScratch t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kTinyBins) t.hist[i] = 0;
    if (i < kTinyClasses) {
        t.counts[i] = 0;
        t.base[i] = 0;
    }
}

// Workgroups take contiguous ranges of pairs (at most kTinyPlanGrid
// workgroups), count them per bin in LDS and add each non-empty bin to the
// global histogram once: a million gaps fall into a few dozen busy bins,
// and one global atomic per bin per workgroup keeps those bins uncontended.
constexpr int kTinyPlanGrid = 512;

RA_DEV void tiny_range(int64_t n_pairs, int64_t &lo, int64_t &hi) {
    const int64_t per = ((n_pairs + gridDim.x - 1) / gridDim.x + kTinyPlanBlock - 1) / kTinyPlanBlock * kTinyPlanBlock;
    lo = (int64_t)blockIdx.x * per;
    hi = lo + per < n_pairs ? lo + per : n_pairs;
}

__global__ __launch_bounds__(kTinyPlanBlock) void k_tiny_count(PairArrays a, int64_t n_pairs, TinyScratch t) {
    __shared__ int h[kTinyBins];
    for (int i = threadIdx.x; i < kTinyBins; i += kTinyPlanBlock) h[i] = 0;
    __syncthreads();
    int64_t lo, hi;
    tiny_range(n_pairs, lo, hi);
    for (int64_t p = lo + threadIdx.x; p < hi; p += kTinyPlanBlock)
        if (tiny_pair(a, p)) atomicAdd(&h[tiny_bin(a.q_len[p], a.r_len[p])], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < kTinyBins; i += kTinyPlanBlock)
        if (h[i]) atomicAdd(&t.hist[i], h[i]);
}

// Exclusive scan of all bins in class-major order (one workgroup of
// kTinyBins threads, Hillis-Steele in LDS): class c then occupies
// list[base[c] .. base[c] + counts[c]).
__global__ __launch_bounds__(kTinyBins) void k_tiny_scan(TinyScratch t) {
    __shared__ int v[kTinyBins];
    const int i = threadIdx.x;
    const int own = t.hist[i];
    v[i] = own;
    __syncthreads();
    for (int off = 1; off < kTinyBins; off <<= 1) {
        const int x = i >= off ? v[i - off] : 0;
        __syncthreads();
        v[i] += x;
        __syncthreads();
    }
    const int excl = v[i] - own;
    t.hist[i] = excl;
    if (i % kTinyBuckets == 0) t.base[i / kTinyBuckets] = excl;
    if (i % kTinyBuckets == kTinyBuckets - 1) {
        const int c = i / kTinyBuckets;
        t.counts[c] = v[i] - (i + 1 - kTinyBuckets == 0 ? 0 : v[i - kTinyBuckets]);
    }
}

// Each workgroup counts its range per bin in LDS, reserves one contiguous
// slot range per bin with a single global atomic on the bin's cursor, then
// ranks its pairs in LDS again and writes them there.
__global__ __launch_bounds__(kTinyPlanBlock) void k_tiny_scatter(PairArrays a, int64_t n_pairs, TinyScratch t) {
    __shared__ int cnt[kTinyBins];
    __shared__ int base[kTinyBins];
    for (int i = threadIdx.x; i < kTinyBins; i += kTinyPlanBlock) cnt[i] = 0;
    __syncthreads();
    int64_t lo, hi;
    tiny_range(n_pairs, lo, hi);
    for (int64_t p = lo + threadIdx.x; p < hi; p += kTinyPlanBlock)
        if (tiny_pair(a, p)) atomicAdd(&cnt[tiny_bin(a.q_len[p], a.r_len[p])], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < kTinyBins; i += kTinyPlanBlock) {
        if (cnt[i]) base[i] = atomicAdd(&t.hist[i], cnt[i]);
        cnt[i] = 0;
    }
    __syncthreads();
    for (int64_t p = lo + threadIdx.x; p < hi; p += kTinyPlanBlock) {
        if (tiny_pair(a, p)) {
            const int bin = tiny_bin(a.q_len[p], a.r_len[p]);
            TinyRec rc;
            rc.q_off = a.q_off[p];
            rc.r_off = a.r_off[p];
            rc.p = (int32_t)p;
            rc.n = a.q_len[p];
            rc.m = a.r_len[p];
            rc.unused = 0;
            t.list[base[bin] + atomicAdd(&cnt[bin], 1)] = rc;
        }
    }
}

// One query row over the lane's W slots.  diag0: north-west value of slot 0
// (the corner at row 0 when m == W, else +inf); west of slot 0 is +inf.
template <int W>
RA_DEV void tiny_row(float qv, float diag0, const float (&rv)[W], const float (&Ao)[W], float (&An)[W]) {
    An[0] = fabsf(qv - rv[0]) + fminf(diag0, Ao[0]);
#pragma unroll
    for (int v = 1; v < W; ++v) An[v] = cell(qv, rv[v], Ao[v - 1], Ao[v], An[v - 1]);
}

// Query events are read kTinyQB rows at a time, one block ahead of use, so
// the per-lane gathers are in flight while the previous block computes.
constexpr int kTinyQB = 8;

template <int W>
RA_DEV void tiny_qblock(const float *qp, int n, int i0, float (&qb)[kTinyQB]) {
#pragma unroll
    for (int k = 0; k < kTinyQB; ++k) qb[k] = qp[i0 + k < n ? i0 + k : n - 1];
}

// Gaps of width class `cls` (m <= W levels), 64 per wave, in list order.
// Narrow classes are bound by the latency of their gathers (the gap record,
// then levels and events), not by their few cells.  W = 12 asks the
// compiler for 6 resident waves per SIMD instead of 5 (at most 80 VGPRs, no
// spills); W = 16 would spill there.  The same request for 8 waves at W <= 8
// made those classes slower.
template <int W>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(W == 12 ? 6 : 1)))
void k_tiny(PairArrays a, TinyScratch t, int cls) {
    const int count = t.counts[cls];
    const TinyRec *list = t.list + t.base[cls];
    const int lane = __lane_id();
    for (int base = blockIdx.x * 64; base < count; base += gridDim.x * 64) {
        const bool act = base + lane < count;
        const TinyRec rc = list[act ? base + lane : count - 1];   // idle lanes repeat the last gap
        const int p = rc.p;
        const int n = rc.n;   // >= 1
        const int m = rc.m;   // 1 .. W
        const float *qp = a.q + rc.q_off;
        const float *rp = a.r + rc.r_off;
        const int pad = W - m;
        // Slot v holds level v - pad; slots left of the gap are never read
        // from memory (the load is masked off for them).
        const float *rs = rp - pad;
        float rv[W], A[W], B[W];
#pragma unroll
        for (int v = 0; v < W; ++v) {
            rv[v] = v >= pad ? rs[v] : kInf;
            A[v] = v == pad - 1 ? 0.0f : kInf;
        }
        float corner = pad == 0 ? 0.0f : kInf;
        int nmax = n;   // the wave runs as long as its longest gap
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) nmax = max(nmax, __shfl_xor(nmax, off, 64));
        float res = kInf;
        float qc[kTinyQB], qn[kTinyQB];
        tiny_qblock<W>(qp, n, 0, qc);
        for (int i0 = 0; i0 < nmax; i0 += kTinyQB) {
            tiny_qblock<W>(qp, n, i0 + kTinyQB, qn);
#pragma unroll
            for (int k = 0; k < kTinyQB; k += 2) {
                tiny_row<W>(qc[k], corner, rv, A, B);
                corner = kInf;
                if (i0 + k == n - 1) res = B[W - 1];
                tiny_row<W>(qc[k + 1], kInf, rv, B, A);
                if (i0 + k + 1 == n - 1) res = A[W - 1];
            }
#pragma unroll
            for (int k = 0; k < kTinyQB; ++k) qc[k] = qn[k];
        }
        if (act) {
            a.out_score[p] = res;
            if (a.out_end) a.out_end[p] = m - 1;
        }
    }
}

// The four widest classes (W = 24 .. 64) take two lanes per gap.  Alone, a
// lane's longest gap sets such a class's time: one instruction chain of
// n x W cells (W = 64, n = 283 on the anchored workload).  Lane 2k holds
// slots [0, W/2) of gap k and lane 2k+1 slots [W/2, W); the second runs one
// row behind and takes the west value of its first slot from its partner's
// last slot of that row (one DPP move per row), its north-west value from
// the row before.  Each chain is half as long, with fewer registers.  Every
// region of these classes has more than W/2 levels, so the pad W - m is
// below W/2 and the corner of row -1 (slot pad - 1) lies in the first half;
// the second lane's row -1 is then all +inf, its first step (on a row
// before the gap) leaves it at +inf, and no step needs to be peeled off.
template <int H>
RA_DEV void tiny_half_row(float qv, float nw0, float w0, const float (&rv)[H], const float (&Ao)[H],
                          float (&An)[H]) {
    An[0] = cell(qv, rv[0], nw0, Ao[0], w0);
#pragma unroll
    for (int v = 1; v < H; ++v) An[v] = cell(qv, rv[v], Ao[v - 1], Ao[v], An[v - 1]);
}

// Rows i0 - half .. i0 - half + kTinyQB - 1 of the lane, clamped to [0, n).
RA_DEV void tiny_qblock_half(const float *qp, int n, int i0, float (&qb)[kTinyQB]) {
#pragma unroll
    for (int k = 0; k < kTinyQB; ++k) {
        const int i = i0 + k;
        qb[k] = qp[i < 0 ? 0 : (i < n ? i : n - 1)];
    }
}

RA_DEV float partner(float x) {   // lane 2k+1 receives lane 2k's value (and 2k receives 2k+1's)
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
}

template <int W>
__global__ __launch_bounds__(64) void k_tiny_pair(PairArrays a, TinyScratch t, int cls) {
    constexpr int H = W / 2;
    const int count = t.counts[cls];
    const TinyRec *list = t.list + t.base[cls];
    const int lane = __lane_id();
    const int half = lane & 1;
    for (int base = blockIdx.x * 32; base < count; base += gridDim.x * 32) {
        const int g = base + (lane >> 1);
        const bool act = g < count;
        const TinyRec rc = list[act ? g : count - 1];   // idle pairs of lanes repeat the last gap
        const int p = rc.p;
        const int n = rc.n;   // >= 1
        const int m = rc.m;   // W/2 < m <= W
        const float *qp = a.q + rc.q_off;
        const float *rs = a.r + rc.r_off - (W - m);
        const int pad = W - m;
        const int v0 = half * H;
        float rv[H], A[H], B[H];
#pragma unroll
        for (int v = 0; v < H; ++v) {
            rv[v] = v0 + v >= pad ? rs[v0 + v] : kInf;
            A[v] = v0 + v == pad - 1 ? 0.0f : kInf;
        }
        float corner = half == 0 && pad == 0 ? 0.0f : kInf;
        int nmax = n;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) nmax = max(nmax, __shfl_xor(nmax, off, 64));
        float res = kInf;
        float mylast = kInf;      // this lane's last slot, previous step
        float edge_prev = kInf;   // the partner's last slot two steps back
        float qc[kTinyQB], qn[kTinyQB];
        tiny_qblock_half(qp, n, -half, qc);
        // step s: the first lane computes row s, the second row s - 1
        for (int i0 = 0; i0 <= nmax; i0 += kTinyQB) {
            tiny_qblock_half(qp, n, i0 + kTinyQB - half, qn);
#pragma unroll
            for (int k = 0; k < kTinyQB; k += 2) {
                float edge = partner(mylast);
                tiny_half_row<H>(qc[k], half ? edge_prev : corner, half ? edge : kInf, rv, A, B);
                corner = kInf;
                edge_prev = edge;
                mylast = B[H - 1];
                if (half && i0 + k == n) res = B[H - 1];
                edge = partner(mylast);
                tiny_half_row<H>(qc[k + 1], half ? edge_prev : kInf, half ? edge : kInf, rv, B, A);
                edge_prev = edge;
                mylast = A[H - 1];
                if (half && i0 + k + 1 == n) res = A[H - 1];
            }
#pragma unroll
            for (int k = 0; k < kTinyQB; ++k) qc[k] = qn[k];
        }
        if (act && half) {
            a.out_score[p] = res;
            if (a.out_end) a.out_end[p] = m - 1;
        }
    }
}

// Classes that take two lanes per gap: every region of such a class is
// wider than the class below it, and that class is at least half as wide,
// so the pad is below W/2 and the corner stays in the first half.  Pairing
// the narrower classes too (down to W = 8) measured the same.
RA_HOST_DEV constexpr bool tiny_paired(int c) { return c >= 4; }
static_assert(tiny_width(3) >= tiny_width(4) / 2 && tiny_width(4) >= tiny_width(5) / 2 &&
                  tiny_width(5) >= tiny_width(6) / 2 && tiny_width(6) >= tiny_width(7) / 2,
              "paired classes need the corner of row -1 in the first lane's half");

template <int C>
static int tiny_occupancy() {
    static int occ = 0;
    if (!occ) {
        int nb = 0;
        if constexpr (tiny_paired(C))
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiny_pair<tiny_width(C)>, 64, 0);
        else
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiny<tiny_width(C)>, 64, 0);
        occ = nb > 0 ? nb : 1;
    }
    return occ;
}

// Widest class first: its longest gaps are the longest serial chains.
template <int C>
static hipError_t launch_tiny_class(const PairArrays &a, int64_t n_pairs, const TinyScratch &t, int cus,
                                    const hipStream_t *st) {
    if constexpr (C >= 0) {
        // no more waves than the pairs could need (64 gaps per wave, 32 when paired)
        const int per = tiny_paired(C) ? 32 : 64;
        const int64_t need = (n_pairs + per - 1) / per;
        const int64_t full = (int64_t)cus * tiny_occupancy<C>();
        const unsigned grid = (unsigned)(need < full ? need : full);
        if constexpr (tiny_paired(C))
            hipLaunchKernelGGL(k_tiny_pair<tiny_width(C)>, dim3(grid), dim3(64), 0, st[(kTinyClasses - 1 - C) % 3],
                               a, t, C);
        else
            hipLaunchKernelGGL(k_tiny<tiny_width(C)>, dim3(grid), dim3(64), 0, st[(kTinyClasses - 1 - C) % 3], a,
                               t, C);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_tiny_class<C - 1>(a, n_pairs, t, cus, st);
    }
    return hipSuccess;
}

hipError_t launch_tiny_plan(const PairArrays &a, int64_t n_pairs, const TinyScratch &t, hipStream_t stream) {
    hipLaunchKernelGGL(k_tiny_zero, dim3((kTinyBins + 255) / 256), dim3(256), 0, stream, t);
    int64_t g64 = (n_pairs + kTinyPlanBlock - 1) / kTinyPlanBlock;
    const unsigned g = (unsigned)(g64 < kTinyPlanGrid ? g64 : kTinyPlanGrid);
    hipLaunchKernelGGL(k_tiny_count, dim3(g), dim3(kTinyPlanBlock), 0, stream, a, n_pairs, t);
    hipLaunchKernelGGL(k_tiny_scan, dim3(1), dim3(kTinyBins), 0, stream, t);
    hipLaunchKernelGGL(k_tiny_scatter, dim3(g), dim3(kTinyPlanBlock), 0, stream, a, n_pairs, t);
    return hipGetLastError();
}

// The width classes go round the three streams, widest first: each class is
// about one round of waves, whose time its longest gaps set, so classes on
// different streams overlap.
hipError_t launch_tiny(const PairArrays &a, int64_t n_pairs, const TinyScratch &t, int cus, const hipStream_t *st) {
    return launch_tiny_class<kTinyClasses - 1>(a, n_pairs, t, cus, st);
}

// ---- chain sums ------------------------------------------------------------------

// Chain c costs the sum of its gaps' costs, added one after another in gap
// order (one float rounding per gap, the same order as a sequential sum).  A
// chain without gaps costs 0; a gap range outside [0, n_gaps) gives NaN.
__global__ void k_chain_sum(const float *__restrict__ gap_cost, int64_t n_gaps,
                            const int64_t *__restrict__ chain_gap_off, const int32_t *__restrict__ chain_gap_cnt,
                            int64_t n_chains, float *__restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chains) return;
    const int64_t g0 = chain_gap_off[c];
    const int cnt = chain_gap_cnt[c];
    if (cnt < 0 || g0 < 0 || g0 + cnt > n_gaps) {
        out[c] = __builtin_nanf("");
        return;
    }
    // Eight gap costs are loaded at a time, so their latencies overlap; the
    // additions still run one after another in gap order.
    float acc = 0.0f;
    for (int g = 0; g < cnt; g += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = g + j < cnt ? gap_cost[g0 + g + j] : 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (g + j < cnt) acc = acc + v[j];
    }
    out[c] = acc;
}

hipError_t launch_chain_sum(const float *gap_cost, int64_t n_gaps, const int64_t *chain_gap_off,
                            const int32_t *chain_gap_cnt, int64_t n_chains, float *out_chain_cost,
                            hipStream_t stream) {
    const unsigned g = (unsigned)((n_chains + 255) / 256);
    hipLaunchKernelGGL(k_chain_sum, dim3(g), dim3(256), 0, stream, gap_cost, n_gaps, chain_gap_off, chain_gap_cnt,
                       n_chains, out_chain_cost);
    return hipGetLastError();
}

}  // namespace ra
