// dtw_bnb.hip -- early termination of hopeless candidates (branch and bound).
//
// RawAlign outputs at most one mapping per read and prunes DTW work that
// cannot beat the best candidate found so far; candidates are visited in
// chaining-score order so that a good one comes first (Sec. 2.4.1).  Here one
// persistent kernel takes the pairs from a queue that holds every read's
// first candidate before all other candidates (longest first within each
// group).  A wave sweeps its pair in blocks of query rows through the pair's
// resident row.  After a block that ended at row i the sweep knows
// min_j D(i, j); every path reaches row n-1 through row i and costs never
// decrease along a path (each cell adds |q - r| >= 0), so
// C_DTW >= min_j D(i, j) and the pair's Score is at most
// B_Match * N_Read - min_j D(i, j).  When that is strictly below the best
// Score its read has reached so far the pair cannot win (nor tie) and the
// wave drops it; a pair that completes raises its read's best with an
// atomic maximum.  The best only grows, so every drop is justified by the
// final best: the read's decision (argmax Score, smallest index on ties,
// threshold) is the one of the full computation, whatever the timing.
#include "dtw_device.h"

namespace ra {

// Monotone encoding of doubles as unsigned 64-bit keys (larger double ->
// larger key), so the per-read best can be raised with an integer atomicMax.
RA_DEV uint64_t order_key(double d) {
    const uint64_t b = __builtin_bit_cast(uint64_t, d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
RA_DEV double order_value(uint64_t k) {
    const uint64_t b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __builtin_bit_cast(double, b);
}

// Pair checks: the same rules as the batch entry point (slices inside q and
// r, region and query limits) plus the row slot and the caller's longest
// query.
RA_DEV bool bnb_valid(const BnbArgs &b, int64_t p) {
    const PairArrays &a = b.a;
    const int n = a.q_len[p];
    const int m = a.r_len[p];
    const int64_t qo = a.q_off[p];
    const int64_t ro = a.r_off[p];
    const int64_t wo = a.row_off[p];
    return n >= 0 && m >= 0 && qo >= 0 && ro >= 0 && qo + n <= a.q_size && ro + m <= a.r_size &&
           m <= kMaxRegion && n <= kMaxQuery && (m <= kSingleMaxRegion || n <= kEdgeCap) && n <= b.max_query &&
           wo >= 0 && wo + m <= a.rows_size;
}

// Per pair: read of the pair (claimed through the reads' candidate ranges),
// status, and results of pairs that need no DTW.
__global__ void k_bnb_clear(BnbArgs b) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < b.n_pairs) {
        b.s.read_of[p] = -1;
        b.s.status[p] = kBnbWaiting;
    }
    if (p < b.n_reads) b.s.best[p] = order_key(-__builtin_inf());
}

__global__ void k_bnb_claim(BnbArgs b) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= b.n_reads) return;
    const int64_t p0 = b.cand_off[k];
    const int cnt = b.cand_cnt[k];
    if (cnt <= 0 || p0 < 0 || p0 + cnt > b.n_pairs) return;   // rawalign_decide flags such reads
    for (int c = 0; c < cnt; ++c) {
        // A pair claimed by two reads is never pruned (it has no single bound).
        if (atomicCAS(&b.s.read_of[p0 + c], -1, (int32_t)k) != -1) atomicExch(&b.s.read_of[p0 + c], -2);
    }
    b.s.status[p0] = kBnbFirst;   // queued ahead of the others (reads own disjoint first pairs)
}

__global__ void k_bnb_prepare(BnbArgs b) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= b.n_pairs) return;
    const PairArrays &a = b.a;
    float sc;
    int e;
    bool done = true;
    if (!bnb_valid(b, p)) {
        sc = __builtin_nanf("");
        e = -2;
    } else if (a.q_len[p] == 0) {
        sc = 0.0f;
        e = -1;
    } else if (a.r_len[p] == 0) {
        sc = kInf;
        e = -1;
    } else {
        done = false;
    }
    if (done) {
        a.out_score[p] = sc;
        a.out_end[p] = e;
        b.s.status[p] = kBnbDone;
    }
}

// ---- queue: first candidates, then the others, each longest first --------

// Stripes of at most 2048 columns (C <= 32 columns per lane) for every
// region; a region of m levels takes S = ceil(m / 2048)
// stripes of 64 C columns, C = 2h, the smallest with S * 64 C >= m.
constexpr int kBnbMaxK = 8;
// Columns per lane in steps of 2: every count from 1 to 32 in one kernel
// would more than quadruple its compile time.
constexpr int kBnbColStep = 2;
RA_DEV void bnb_shape(int m, int &S, int &h) {
    const int width = 256 * kBnbMaxK;
    S = (m + width - 1) / width;
    if (S < 1) S = 1;
    h = (m + 64 * kBnbColStep * S - 1) / (64 * kBnbColStep * S);
}

// Group (0 first candidates, 1 others) and LPT bucket of pair p, or -1 when
// the pair needs no sweep.
RA_DEV int bnb_bin(const BnbArgs &b, int64_t p) {
    const uint8_t st = b.s.status[p];
    if (st != kBnbFirst && st != kBnbWaiting) return -1;
    const int n = b.a.q_len[p];
    int S, h;
    bnb_shape(b.a.r_len[p], S, h);
    const float work = (float)(n + 64) * (float)(S * 64 * kBnbColStep * h) + 1.0f;
    int k = (int)(4.0f * __log2f(work));
    k = k < 0 ? 0 : (k >= kBuckets ? kBuckets - 1 : k);
    return (st == kBnbFirst ? 0 : kBuckets) + (kBuckets - 1 - k);
}

constexpr int kBnbBins = 2 * kBuckets;

__global__ void k_bnb_zero(BnbArgs b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kBnbBins) b.s.hist[i] = 0;
    if (i < 2) b.s.counts[i] = 0;
    if (i == 0) *b.s.queue = 0;
}

__global__ __launch_bounds__(256) void k_bnb_count(BnbArgs b) {
    __shared__ int h[kBnbBins];
    for (int i = threadIdx.x; i < kBnbBins; i += 256) h[i] = 0;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < b.n_pairs) {
        const int bin = bnb_bin(b, p);
        if (bin >= 0) atomicAdd(&h[bin], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBnbBins; i += 256)
        if (h[i]) atomicAdd(&b.s.hist[i], h[i]);
}

__global__ void k_bnb_scan(BnbArgs b) {
    if (threadIdx.x != 0) return;
    int run = 0;
    for (int g = 0; g < 2; ++g) {
        const int start = run;
        for (int k = 0; k < kBuckets; ++k) {
            const int c = b.s.hist[g * kBuckets + k];
            b.s.hist[g * kBuckets + k] = run;
            run += c;
        }
        b.s.counts[g] = run - start;
    }
}

__global__ __launch_bounds__(256) void k_bnb_scatter(BnbArgs b) {
    __shared__ int cnt[kBnbBins];
    __shared__ int base[kBnbBins];
    for (int i = threadIdx.x; i < kBnbBins; i += 256) cnt[i] = 0;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bin = -1, rank = 0;
    if (p < b.n_pairs) {
        bin = bnb_bin(b, p);
        if (bin >= 0) rank = atomicAdd(&cnt[bin], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBnbBins; i += 256)
        if (cnt[i]) base[i] = atomicAdd(&b.s.hist[i], cnt[i]);
    __syncthreads();
    if (bin >= 0) b.s.list[base[bin] + rank] = (int32_t)p;
}

// ---- the sweep -------------------------------------------------------------------

template <int H>
RA_DEV void bnb_dispatch(int h, const PairView &pv, int S, float *edge, float &best, int &bj) {
    if constexpr (H <= 4 * kBnbMaxK / kBnbColStep) {
        if (h == H)
            multi_pair<kBnbColStep * H, true>(pv, S, edge, best, bj);
        else
            bnb_dispatch<H + 1>(h, pv, S, edge, best, bj);
    }
}

// Wave priority (0..3) while sweeping a read's first candidate.
#ifndef RA_BNB_FIRST_PRIO
#define RA_BNB_FIRST_PRIO 0
#endif
constexpr int kBnbFirstPrio = RA_BNB_FIRST_PRIO;

RA_DEV int bnb_next(int32_t *queue) {
    int it = 0;
    if (__lane_id() == 0) it = atomicAdd(queue, 1);
    return __builtin_amdgcn_readfirstlane(it);
}

// Three waves per SIMD: at four, every column count from 2 to 32 in one
// kernel plus the block loop spill registers.
#ifndef RA_BNB_WAVES
#define RA_BNB_WAVES 3
#endif
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(RA_BNB_WAVES, RA_BNB_WAVES)))
void k_bnb_run(BnbArgs b, float *edge_base) {
    float *edge = edge_base + (size_t)blockIdx.x * kEdgeCap;
    const PairArrays &a = b.a;
    const int n_items = b.s.counts[0] + b.s.counts[1];
    int item = bnb_next(b.s.queue);
    while (item < n_items) {
        const int p = b.s.list[item];
        // First candidates carry the longest dependency chains (their
        // reads' bounds and, longest first, the kernel's critical path).
        if (kBnbFirstPrio > 0) {
            if (item < b.s.counts[0])
                __builtin_amdgcn_s_setprio(kBnbFirstPrio);
            else
                __builtin_amdgcn_s_setprio(0);
        }
        PairView pv;
        pv.q = a.q + a.q_off[p];
        pv.n = a.q_len[p];
        pv.r = a.r + a.r_off[p];
        pv.m = a.r_len[p];
        pv.row = a.rows + a.row_off[p];
        pv.corner = false;    // subsequence alignment, forward
        pv.fixed_end = false;
        pv.reverse = false;
        const int n = pv.n;   // >= 1, m >= 1 (others were settled before)
        int S, h;
        bnb_shape(pv.m, S, h);
        float best = kInf;
        int bj = 0x7fffffff;
        bool pruned = false;
        for (int row0 = 0; row0 < n; row0 += b.block_rows) {
            PairView pb = pv;
            pb.q = pv.q + row0;
            pb.n = n - row0 < b.block_rows ? n - row0 : b.block_rows;
            pb.fresh = row0 == 0;
            bnb_dispatch<1>(h, pb, S, edge, best, bj);
            if (row0 + pb.n >= n) continue;
            // Bound check (values reloaded here rather than kept live across
            // the sweep); one address, so one value for the wave.
            const int k = __builtin_amdgcn_readfirstlane(b.s.read_of[p]);
            if (k < 0) continue;
            const uint64_t key = __hip_atomic_load(&b.s.best[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)key);
            const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(key >> 32));
            const double cur = order_value(((uint64_t)hi << 32) | lo);
            if (b.b_match * (double)b.n_events[k] - (double)best < cur) {
                pruned = true;
                break;
            }
        }
        if (__lane_id() == 0) {
            if (pruned) {
                a.out_score[p] = kInf;   // cannot win: treated as unmapped by the decision
                a.out_end[p] = -3;
            } else {
                a.out_score[p] = best;
                a.out_end[p] = bj;
                const int k = b.s.read_of[p];
                if (k >= 0)
                    atomicMax((unsigned long long *)&b.s.best[k],
                              (unsigned long long)order_key(b.b_match * (double)b.n_events[k] - (double)best));
            }
        }
        item = bnb_next(b.s.queue);
    }
}

static unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_bnb(const BnbArgs &b, int grid, float *edge, hipStream_t stream) {
    const int64_t mx = b.n_pairs > b.n_reads ? b.n_pairs : b.n_reads;
    hipLaunchKernelGGL(k_bnb_clear, dim3(grid_of(mx)), dim3(256), 0, stream, b);
    hipLaunchKernelGGL(k_bnb_claim, dim3(grid_of(b.n_reads)), dim3(256), 0, stream, b);
    hipLaunchKernelGGL(k_bnb_prepare, dim3(grid_of(b.n_pairs)), dim3(256), 0, stream, b);
    hipLaunchKernelGGL(k_bnb_zero, dim3(grid_of(kBnbBins)), dim3(256), 0, stream, b);
    hipLaunchKernelGGL(k_bnb_count, dim3(grid_of(b.n_pairs)), dim3(256), 0, stream, b);
    hipLaunchKernelGGL(k_bnb_scan, dim3(1), dim3(64), 0, stream, b);
    hipLaunchKernelGGL(k_bnb_scatter, dim3(grid_of(b.n_pairs)), dim3(256), 0, stream, b);
    hipLaunchKernelGGL(k_bnb_run, dim3((unsigned)grid), dim3(64), 0, stream, b, edge);
    return hipGetLastError();
}

int bnb_blocks_per_cu() {
    int nb = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bnb_run, 64, 0);
    return nb > 0 ? nb : 1;
}

}  // namespace ra
