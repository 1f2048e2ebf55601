// Internal interface between the C ABI (rawalign_abi.cpp) and the kernels
// (dtw_single.hip, dtw_multi.hip, dtw_antidiag.hip, dtw_plan.hip, dtw_bnb.hip).  Not installed; the public
// interface is include/rawalign.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ra {

#define RA_HOST_DEV __host__ __device__

// Routes a pair can take after planning:
//   single_lo: one stripe, 2..32 columns per lane (region <= 2048 levels)
//   single_hi: one stripe, 34..64 columns per lane (region <= 4096 levels)
//   multi:     several stripes of at most 256 kMultiMaxK columns swept one
//              after another by the same wave (region > 4096 levels)
// The banded planner (dtw_plan.hip, band mode) uses the same lists for its
// four pair classes, so there are four lists although plain batches use
// three.
enum Route : int { kRouteSingleLo = 0, kRouteSingleHi = 1, kRouteMulti = 2, kNumRoutes = 4 };
constexpr int kNumBandClasses = 4;

constexpr int kMaxColsPerLane = 64;
constexpr int kShortMaxRegion = 64 * kMaxColsPerLane;  // 4096: the widest single stripe
constexpr int kSingleLoMaxRegion = 2048;               // 64 lanes x 32 columns
constexpr int kMaxStripes = 16;
constexpr int kMaxRegion = kMaxStripes * kShortMaxRegion;   // 65536
// Columns per lane come in steps (C = step * h).  Single-stripe kernels use
// steps of 2 (32 column counts per kernel).  The multi-stripe and
// early-termination kernels use steps of 1 by default, which halves the
// padding columns past the end of a region; the two-chain sweep needs 2.
constexpr int kSingleColStep = 2;
#ifndef RA_MULTI_COL_STEP
#define RA_MULTI_COL_STEP 1
#endif
constexpr int kMultiColStep = RA_MULTI_COL_STEP;
static_assert(kMultiColStep == 1 || kMultiColStep == 2, "column step");

// Widest region the single-stripe kernel takes, in groups of 4 columns per
// lane (16: 4096 levels at two waves per SIMD; 11: 2816 levels at three).
#ifndef RA_SINGLE_HI_KMAX
#define RA_SINGLE_HI_KMAX 16
#endif
constexpr int kSingleHiMaxK = RA_SINGLE_HI_KMAX;
constexpr int kSingleMaxRegion = 256 * kSingleHiMaxK;
static_assert(kSingleHiMaxK >= 8 && kSingleHiMaxK <= 16, "single-stripe width");
// Widest stripe of the multi-stripe kernel, in groups of 4 columns per lane
// (16: 4096 columns at two waves per SIMD; 8: 2048 columns at four waves per
// SIMD, which issues faster despite the extra stripe boundaries).
#ifndef RA_MULTI_KMAX
#define RA_MULTI_KMAX 8
#endif
constexpr int kMultiMaxK = RA_MULTI_KMAX;
static_assert(kMultiMaxK >= 5 && kMultiMaxK <= 16, "multi-stripe width");
constexpr int kMaxQuery = 1 << 28;                     // keeps 4*n and the step counter in int
constexpr int kEdgeCap = 16384;                        // longest query of a multi-stripe pair

// Number of LPT buckets per route: cells are bucketed by quarter octaves.
constexpr int kBuckets = 192;

// Per-stream planning scratch (device memory).
struct PlanScratch {
    int32_t *hist;      // [kNumRoutes * kBuckets] histogram, then cursors
    int32_t *counts;    // [kNumRoutes]  pairs per route
    int32_t *queue;     // [kNumRoutes]  persistent work-queue heads
    int32_t *list;      // [kNumRoutes * capacity] pair indices per route
    int64_t capacity;   // pairs the lists can hold
    float *edge;        // [multi_grid * kEdgeCap] stripe edge columns, one slot per wave
    float *rowbuf;      // [antidiag_grid * kMaxRegion] anti-diagonal kernel row buffers (or null)
};

struct PairArrays {
    const float *q;
    int64_t q_size;
    const int64_t *q_off;
    const int32_t *q_len;
    const float *r;
    int64_t r_size;
    const int64_t *r_off;
    const int32_t *r_len;
    float *out_score;
    int32_t *out_end;
    // streaming extension (null for plain batches)
    float *rows;
    int64_t rows_size;
    const int64_t *row_off;
    const uint8_t *first_chunk;
    // Boundary and result (BoundMode): subsequence, global between anchors,
    // or anchored start with a free end.
    int bound = 0;
    // 1: read query and region back to front: query element t is
    // q[n-1-t], region column j is r[m-1-j].
    int reverse = 0;
};

// Boundary and result of an alignment:
//   kBoundSubseq:   row -1 zero (free start), C = min of the last row;
//   kBoundGlobal:   global between two anchors (Sec. 2.4.2): the path enters
//                   at (0, 0) from the corner D(-1,-1) = 0, the rest of row
//                   -1 is +inf, and the result is D(n-1, m-1);
//   kBoundAnchored: the corner boundary with the subsequence result: the
//                   reverse pass that finds where an alignment starts.
enum BoundMode : int { kBoundSubseq = 0, kBoundGlobal = 1, kBoundAnchored = 2 };

// Global pairs of at most kTinyMaxCols levels are aligned one pair per lane
// (dtw_global.hip); the planning of the striped kernels leaves them out.
constexpr int kTinyClasses = 8;
constexpr int kTinyMaxCols = 64;
constexpr int kTinyBuckets = 128;   // quarter octaves of the query length
RA_HOST_DEV constexpr int tiny_width(int c) {
    return c == 0 ? 4 : c == 1 ? 8 : c == 2 ? 12 : c == 3 ? 16 : c == 4 ? 24 : c == 5 ? 32 : c == 6 ? 48 : 64;
}

// One gap of the one-lane kernel's list: its pair index and what the kernel
// reads of it, so a lane starts with one coalesced 32-byte load instead of
// a list entry and then four gathers that depend on it.
struct alignas(16) TinyRec {
    int64_t q_off;
    int64_t r_off;
    int32_t p;
    int32_t n;
    int32_t m;
    int32_t unused;
};

struct TinyScratch {
    int32_t *hist;      // [kTinyClasses * kTinyBuckets] histogram, then cursors
    int32_t *counts;    // [kTinyClasses] pairs per width class
    int32_t *base;      // [kTinyClasses] first list slot of each class
    TinyRec *list;      // [capacity] gaps, class by class, longest queries first
    int64_t capacity;
};

// Early termination (branch and bound): pair status and scratch.
enum BnbStatus : uint8_t { kBnbWaiting = 0, kBnbFirst = 1, kBnbDone = 2 };

struct BnbScratch {
    int32_t *read_of;     // [n_pairs] read owning the pair, -1 none, -2 several
    uint8_t *status;      // [n_pairs] BnbStatus
    uint64_t *best;       // [n_reads] best Score so far, order-preserving key
    int32_t *list;        // [n_pairs] pairs to align: first candidates, then the others, longest first
    int32_t *hist;        // [2 * kBuckets] histogram, then cursors
    int32_t *counts;      // [2] pairs per group
    int32_t *queue;       // work-queue head
};

struct BnbArgs {
    PairArrays a;         // pairs, resident rows and final outputs
    int64_t n_pairs;
    const int64_t *cand_off;
    const int32_t *cand_cnt;
    const int32_t *n_events;
    int64_t n_reads;
    double b_match;
    int max_query;
    int block_rows;
    BnbScratch s;
};

struct LaunchCfg {
    bool persistent;    // atomic queue + LPT order (else static assignment, arrival order)
    int lo_grid;        // grid sizes (workgroups of one wave)
    int hi_grid;
    int multi_grid;     // workgroups of the multi-stripe route (one wave, or pipe_waves in the pipeline); also
                        // the number of edge slots
    int antidiag_grid;  // workgroups of the anti-diagonal kernel (256 threads)
    int single_max = kSingleMaxRegion;   // widest region of the single-stripe routes (2048 or 4096)
};

// Waves sharing a pair in the pipelined multi-stripe kernel (dtw_pipe.hip).
constexpr int kPipeMaxWaves = 8;

hipError_t launch_plan(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg,
                       const PlanScratch &s, hipStream_t stream);
hipError_t launch_single_lo(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg,
                            const PlanScratch &s, hipStream_t stream);
hipError_t launch_single_hi(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg,
                            const PlanScratch &s, hipStream_t stream);
hipError_t launch_multi(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg,
                        const PlanScratch &s, hipStream_t stream);
hipError_t launch_antidiag(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg,
                           const PlanScratch &s, hipStream_t stream);
// Multi-stripe route on workgroups of `waves` waves (2, 4 or 8) sharing each
// pair, stripes pipelined (dtw_pipe.hip).
hipError_t launch_pipe(int waves, const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg,
                       const PlanScratch &s, hipStream_t stream);
int pipe_blocks_per_cu(int waves, bool extend);
hipError_t launch_bnb(const BnbArgs &b, int grid, float *edge, hipStream_t stream);
int bnb_blocks_per_cu();
// per_candidate: n_events holds one count per candidate (anchored chains)
// instead of one per read.
hipError_t launch_decide(const float *score, int64_t n_pairs, const int64_t *cand_off, const int32_t *cand_cnt,
                         const int32_t *n_events, int64_t n_reads, double b_match, double threshold,
                         int32_t *out_best, double *out_score, uint8_t *out_mapped, bool per_candidate,
                         hipStream_t stream);
hipError_t launch_tiny_plan(const PairArrays &a, int64_t n_pairs, const TinyScratch &t, hipStream_t stream);
hipError_t launch_tiny(const PairArrays &a, int64_t n_pairs, const TinyScratch &t, int cus,
                       const hipStream_t *streams);
// Alignment start: the reverse pass's region lengths (end + 1) and, after
// it, start = end - (reverse pass end).
hipError_t launch_span_prep(const int32_t *end, int64_t n_pairs, int32_t *rev_len, hipStream_t stream);
hipError_t launch_span_finish(const int32_t *end, const int32_t *rev_end, int64_t n_pairs, int32_t *out_start,
                              hipStream_t stream);
// Banded subsequence DTW, one wave per pair.  The planner (same scratch and
// kernels as the striped routes) gives every pair a band class (two frame
// widths of the band-relative kernel, and the whole-region kernel for the
// shapes it does not take) and writes the sentinels of the pairs that need
// no kernel; each class kernel then takes its list longest first from its
// persistent queue.
constexpr int kBandMaxFrame = 64 * 32;   // band columns one wave takes (C <= 32 per lane)
constexpr int kBandLoMaxH = 4;           // class 0: frames of at most 4*128 columns (C <= 8)
hipError_t launch_band_plan(const PairArrays &a, const int32_t *band, int64_t n_pairs, const PlanScratch &s,
                            hipStream_t stream);
hipError_t launch_band(int cls, const PairArrays &a, const int32_t *band, int grid, const PlanScratch &s,
                       hipStream_t stream);
int band_blocks_per_cu(int cls);
hipError_t launch_chain_sum(const float *gap_cost, int64_t n_gaps, const int64_t *chain_gap_off,
                            const int32_t *chain_gap_cnt, int64_t n_chains, float *out_chain_cost,
                            hipStream_t stream);

// Allocation-free batch (rawalign_dtw_batch_noalloc): planning words, pair
// lists for at most kNoallocMaxPairs pairs and kNoallocEdgeSlots stripe-edge
// slots (so at most that many resident multi-stripe waves) in one fixed
// device array per GPU (dtw_noalloc.hip).  noalloc_scratch looks up the
// calling device's copy (once per device, with that device current) and
// returns its views; it allocates nothing.
constexpr int64_t kNoallocMaxPairs = 1 << 17;
constexpr int kNoallocEdgeSlots = 512;
constexpr size_t kNoallocScratchBytes =
    ((sizeof(int32_t) * ((size_t)kNumRoutes * kBuckets + 2 * kNumRoutes) + 255) / 256 * 256) +
    ((sizeof(int32_t) * (size_t)kNumRoutes * kNoallocMaxPairs + 255) / 256 * 256) +
    sizeof(float) * (size_t)kNoallocEdgeSlots * kEdgeCap;
hipError_t noalloc_scratch(int dev, PlanScratch &out);

// Occupancy-derived resident workgroups per CU of each route's kernel.
int single_lo_blocks_per_cu(bool extend);
int single_hi_blocks_per_cu(bool extend);
int multi_blocks_per_cu(bool extend);
int antidiag_blocks_per_cu();

}  // namespace ra
