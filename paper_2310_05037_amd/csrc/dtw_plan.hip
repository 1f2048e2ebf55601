// dtw_plan.hip -- device-side planning (routing, longest-first ordering,
// sentinels for degenerate or invalid pairs) and the mapping decision.
#include "dtw_device.h"

namespace ra {

struct PlanArgs {
    PairArrays a;
    int64_t n_pairs;
    int buckets;      // 1: single bucket (plain), kBuckets: LPT buckets
    int extend;
    int single_max;   // widest region of the single-stripe routes
    PlanScratch s;
    const int32_t *band;   // banded planning (band half-width per pair), else null
};

// Banded pairs (dtw_band.hip): class 0 for frames of at most kBandLoMaxH*128
// columns, class 1 for wider ones, longest first by the frame cells swept;
// for the shapes the band-relative frame does not take (more levels than
// events, or a band wider than one wave's frame), class 2 when the whole
// region fits one wave's frame and class 3 (stripes) above that.  Pairs
// that need no kernel get their result here: NaN/-2 for an invalid slice
// or a negative band, (0, -1) for an empty query, (+inf, -1) for an empty
// region, NaN/-4 for the one shape left: a query longer than a stripe edge
// column (kEdgeCap) against more than 2048 levels with a band wider than
// 2048 columns.
RA_DEV int band_classify(const PlanArgs &pa, int64_t p, int &bucket, float &score, int &end) {
    const PairArrays &a = pa.a;
    const int n = a.q_len[p];
    const int m = a.r_len[p];
    const int wraw = pa.band[p];
    if (!slices_ok(a, p, false) || wraw < 0) {
        score = __builtin_nanf("");
        end = -2;
        return -1;
    }
    if (n == 0 || m == 0) {
        score = n == 0 ? 0.0f : kInf;
        end = -1;
        return -1;
    }
    const int w = wraw < m - 1 ? wraw : m - 1;
    const int W = 2 * w + 1;
    if (m > n || W > kBandMaxFrame) {
        if (m <= kBandMaxFrame) {
            const float work = (float)(n + 64) * (float)(128 * ((m + 127) / 128)) + 1.0f;
            int b = (int)(4.0f * __log2f(work));
            b = b < 0 ? 0 : (b >= kBuckets ? kBuckets - 1 : b);
            bucket = kBuckets - 1 - b;
            return 2;
        }
        if (n <= kEdgeCap) {
            // stripes of the band's rows only: about the rows the band
            // spends in each stripe times its width
            int S, h;
            const int cols = stripe_shape(m, S, h, false);
            const float rows = fminf((float)n, (float)(cols + W) * (float)n / (float)m + 64.0f);
            const float work = rows * (float)(S * cols) + 1.0f;
            int b = (int)(4.0f * __log2f(work));
            b = b < 0 ? 0 : (b >= kBuckets ? kBuckets - 1 : b);
            bucket = kBuckets - 1 - b;
            return 3;
        }
        score = __builtin_nanf("");
        end = -4;
        return -1;
    }
    const int h = (W + 127) / 128;
    const float work = (float)(n + 64) * (float)(128 * h) + 1.0f;
    int b = (int)(4.0f * __log2f(work));
    b = b < 0 ? 0 : (b >= kBuckets ? kBuckets - 1 : b);
    bucket = kBuckets - 1 - b;
    return h <= kBandLoMaxH ? 0 : 1;
}

// Route of pair p.  Returns -1 when the pair needs no kernel; then
// (score, end) is its result: a sentinel for invalid slices (NaN, -2) or the
// value of a degenerate pair (empty query or empty region).  Returns -2 for
// a global pair that the one-pair-per-lane kernel aligns (no output here).
RA_DEV int classify(const PlanArgs &pa, int64_t p, int &bucket, float &score, int &end) {
    if (pa.band) return band_classify(pa, p, bucket, score, end);
    const PairArrays &a = pa.a;
    const int n = a.q_len[p];
    const int m = a.r_len[p];
    const bool ok = slices_ok(a, p, pa.extend != 0);
    const bool fresh = pa.extend ? a.first_chunk[p] != 0 : true;
    if (!ok) {
        score = __builtin_nanf("");
        end = -2;
        return -1;
    }
    if (a.bound == kBoundGlobal) {
        // Anchors touching diagonally cost 0; a gap with events but no
        // levels (or levels but no events) has no path: +inf.
        if (n == 0 || m == 0) {
            score = (n == 0 && m == 0) ? 0.0f : kInf;
            end = -1;
            return -1;
        }
        if (m <= kTinyMaxCols && !a.reverse) return -2;
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
    // Single-stripe routes up to the cut-off; regions up to the widest
    // single stripe whose query is too long for a stripe edge column keep
    // one stripe whatever the cut-off, so the result never depends on it.
    int route;
    if (m <= kSingleLoMaxRegion) route = kRouteSingleLo;
    else if (m <= pa.single_max || (m <= kSingleMaxRegion && n > kEdgeCap)) route = kRouteSingleHi;
    else route = kRouteMulti;
    bucket = 0;
    if (pa.buckets > 1) {
        // Longest-processing-time order: quarter-octave buckets of the swept
        // cells (n + 64 steps per stripe x the stripe's padded columns),
        // bucket 0 holding the largest pairs.
        int S, h;
        const int cols = stripe_shape(m, S, h, route != kRouteMulti);
        const float work = (float)(n + 64) * (float)(S * cols) + 1.0f;
        int b = (int)(4.0f * __log2f(work));
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

// 1024 threads: each thread classifies a few pairs of a million-pair batch,
// one after another; at 256 threads that chain of dependent loads set the
// planning time.
constexpr int kPlanBlock = 1024;
constexpr int kBins = kNumRoutes * kBuckets;
// Workgroups take contiguous ranges of pairs; at most kPlanGrid of them, so
// a batch of millions of pairs still adds each busy bin to the global
// histogram only a few hundred times.
constexpr int kPlanGrid = 512;

RA_DEV void plan_range(int64_t n_pairs, int64_t &lo, int64_t &hi) {
    const int64_t per = ((n_pairs + gridDim.x - 1) / gridDim.x + kPlanBlock - 1) / kPlanBlock * kPlanBlock;
    lo = (int64_t)blockIdx.x * per;
    hi = lo + per < n_pairs ? lo + per : n_pairs;
}

// Each workgroup counts its pairs per (route, bucket) in LDS and adds the
// non-zero bins to the global histogram: one global atomic per bin per
// workgroup instead of one per pair.  Pairs that need no kernel get their
// result here.
__global__ __launch_bounds__(kPlanBlock) void k_plan_count(PlanArgs pa) {
    __shared__ int h[kBins];
    for (int i = threadIdx.x; i < kBins; i += kPlanBlock) h[i] = 0;
    __syncthreads();
    int64_t lo, hi;
    plan_range(pa.n_pairs, lo, hi);
    for (int64_t p = lo + threadIdx.x; p < hi; p += kPlanBlock) {
        int b = 0, e = 0;
        float sc = 0.0f;
        const int route = classify(pa, p, b, sc, e);
        if (route >= 0) {
            atomicAdd(&h[route * kBuckets + b], 1);
        } else if (route == -1) {
            pa.a.out_score[p] = sc;
            if (pa.a.out_end) pa.a.out_end[p] = e;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += kPlanBlock)
        if (h[i]) atomicAdd(&pa.s.hist[i], h[i]);
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

// Each workgroup counts its range per bin in LDS, reserves one contiguous
// range per bin with a single global atomic on the bin's cursor, then ranks
// its pairs in LDS again and writes them there (in plain mode, one bin per
// route: workgroups keep their order of arrival at the cursor, pairs inside
// a workgroup their LDS rank).
__global__ __launch_bounds__(kPlanBlock) void k_plan_scatter(PlanArgs pa) {
    __shared__ int cnt[kBins];
    __shared__ int base[kBins];
    for (int i = threadIdx.x; i < kBins; i += kPlanBlock) cnt[i] = 0;
    __syncthreads();
    int64_t lo, hi;
    plan_range(pa.n_pairs, lo, hi);
    for (int64_t p = lo + threadIdx.x; p < hi; p += kPlanBlock) {
        int b = 0, e = 0;
        float sc = 0.0f;
        const int route = classify(pa, p, b, sc, e);
        if (route >= 0) atomicAdd(&cnt[route * kBuckets + b], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += kPlanBlock) {
        if (cnt[i]) base[i] = atomicAdd(&pa.s.hist[i], cnt[i]);
        cnt[i] = 0;
    }
    __syncthreads();
    for (int64_t p = lo + threadIdx.x; p < hi; p += kPlanBlock) {
        int b = 0, e = 0;
        float sc = 0.0f;
        const int route = classify(pa, p, b, sc, e);
        if (route >= 0) {
            const int bin = route * kBuckets + b;
            pa.s.list[route * pa.s.capacity + base[bin] + atomicAdd(&cnt[bin], 1)] = (int32_t)p;
        }
    }
}

static hipError_t run_plan(const PlanArgs &pa, hipStream_t stream) {
    const PlanScratch &s = pa.s;
    const int64_t n_pairs = pa.n_pairs;
    hipLaunchKernelGGL(k_plan_zero, dim3((kBins + 255) / 256), dim3(256), 0, stream, s);
    const int64_t g64 = (n_pairs + kPlanBlock - 1) / kPlanBlock;
    const unsigned g = (unsigned)(g64 < kPlanGrid ? g64 : kPlanGrid);
    hipLaunchKernelGGL(k_plan_count, dim3(g), dim3(kPlanBlock), 0, stream, pa);
    hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(64), 0, stream, s);
    hipLaunchKernelGGL(k_plan_scatter, dim3(g), dim3(kPlanBlock), 0, stream, pa);
    return hipGetLastError();
}

hipError_t launch_plan(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                       hipStream_t stream) {
    PlanArgs pa;
    pa.a = a;
    pa.n_pairs = n_pairs;
    pa.buckets = cfg.persistent ? kBuckets : 1;
    pa.extend = a.rows != nullptr;
    pa.single_max = cfg.single_max;
    pa.s = s;
    pa.band = nullptr;
    return run_plan(pa, stream);
}

hipError_t launch_band_plan(const PairArrays &a, const int32_t *band, int64_t n_pairs, const PlanScratch &s,
                            hipStream_t stream) {
    PlanArgs pa;
    pa.a = a;
    pa.n_pairs = n_pairs;
    pa.buckets = kBuckets;
    pa.extend = 0;
    pa.single_max = kSingleMaxRegion;
    pa.s = s;
    pa.band = band;
    return run_plan(pa, stream);
}

// ---- alignment start -------------------------------------------------------------

// The reverse pass aligns the reversed query against the reversed region
// prefix r[0 .. end]: end + 1 levels (none for a pair without an end).
__global__ void k_span_prep(const int32_t *__restrict__ end, int64_t n_pairs, int32_t *__restrict__ rev_len) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n_pairs) rev_len[p] = end[p] >= 0 ? end[p] + 1 : 0;
}

// Its best end k (smallest on ties) is the forward column end - k: the
// latest start among the optimal paths ending at end.  Pairs without an
// end keep their sentinel (-1 degenerate, -2 invalid).
__global__ void k_span_finish(const int32_t *__restrict__ end, const int32_t *__restrict__ rev_end, int64_t n_pairs,
                              int32_t *__restrict__ out_start) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n_pairs) out_start[p] = end[p] >= 0 ? end[p] - rev_end[p] : end[p];
}

hipError_t launch_span_prep(const int32_t *end, int64_t n_pairs, int32_t *rev_len, hipStream_t stream) {
    const unsigned g = (unsigned)((n_pairs + 255) / 256);
    hipLaunchKernelGGL(k_span_prep, dim3(g), dim3(256), 0, stream, end, n_pairs, rev_len);
    return hipGetLastError();
}

hipError_t launch_span_finish(const int32_t *end, const int32_t *rev_end, int64_t n_pairs, int32_t *out_start,
                              hipStream_t stream) {
    const unsigned g = (unsigned)((n_pairs + 255) / 256);
    hipLaunchKernelGGL(k_span_finish, dim3(g), dim3(256), 0, stream, end, rev_end, n_pairs, out_start);
    return hipGetLastError();
}

// ---- mapping decision (Sec. 2.3) ----------------------------------------------

// One wave per read.  Score = B_Match * N_Read - C_DTW; the highest wins,
// the smallest candidate index on ties.  Anchored chains count the events
// each chain aligns.  A NaN cost (the sentinel of a pair that was not
// aligned: invalid slice, unsupported shape) is no candidate at all, so it
// can neither win nor block a later candidate.  Lane l scans candidates l,
// l + 64, ... in order and keeps its first highest; the wave then keeps the
// highest score and, among equal scores, the smallest index.  With B_Match
// finite (checked by every entry point) no score is NaN, so this is the
// candidate a sequential first-highest scan picks.
__global__ __launch_bounds__(256) void k_decide(const float *__restrict__ score, int64_t n_pairs,
                                                const int64_t *__restrict__ cand_off,
                                                const int32_t *__restrict__ cand_cnt,
                                                const int32_t *__restrict__ n_events, int64_t n_reads,
                                                double b_match, double threshold, int32_t *out_best,
                                                double *out_score, uint8_t *out_mapped, bool per_candidate) {
    const int lane = __lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; k < n_reads; k += waves) {
        const int64_t p0 = cand_off[k];   // wave-uniform from here on
        const int cnt = cand_cnt[k];
        if (cnt < 0 || p0 < 0 || p0 + cnt > n_pairs) {   // candidate range outside the score array
            if (lane == 0) {
                out_best[k] = -2;
                out_score[k] = __builtin_nan("");
                out_mapped[k] = 0;
            }
            continue;
        }
        const double bonus = per_candidate ? 0.0 : b_match * (double)n_events[k];
        int32_t best = -1;
        double bs = -__builtin_inf();
        for (int c = lane; c < cnt; c += 64) {
            const float cost = score[p0 + c];
            if (cost != cost) continue;
            const double s = (per_candidate ? b_match * (double)n_events[p0 + c] : bonus) - (double)cost;
            if (best < 0 || s > bs) {
                best = (int32_t)(p0 + c);
                bs = s;
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double os = __shfl_xor(bs, off, 64);
            const int32_t ob = __shfl_xor(best, off, 64);
            if (ob >= 0 && (best < 0 || os > bs || (os == bs && ob < best))) {
                best = ob;
                bs = os;
            }
        }
        if (lane == 0) {
            out_best[k] = best;
            out_score[k] = bs;
            out_mapped[k] = (best >= 0 && bs >= threshold) ? 1 : 0;
        }
    }
}

hipError_t launch_decide(const float *score, int64_t n_pairs, const int64_t *cand_off, const int32_t *cand_cnt,
                         const int32_t *n_events, int64_t n_reads, double b_match, double threshold,
                         int32_t *out_best, double *out_score, uint8_t *out_mapped, bool per_candidate,
                         hipStream_t stream) {
    // four waves (one read each at a time) per workgroup
    const int64_t g64 = (n_reads + 3) / 4;
    const unsigned g = (unsigned)(g64 < (1 << 20) ? g64 : (1 << 20));
    hipLaunchKernelGGL(k_decide, dim3(g), dim3(256), 0, stream, score, n_pairs, cand_off, cand_cnt, n_events,
                       n_reads, b_match, threshold, out_best, out_score, out_mapped, per_candidate);
    return hipGetLastError();
}

}  // namespace ra
