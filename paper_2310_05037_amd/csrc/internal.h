// Internal interface between the C ABI (rawalign_abi.cpp) and the kernels
// (dtw_kernels.hip).  Not installed; the public interface is include/rawalign.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ra {

// Routes a pair can take after planning.
// short (lo/hi): one wave per pair, at most / more than 32 columns per lane;
// long: `coop_waves` cooperating waves; huge: the region needs more columns
// than `coop_waves` waves hold, so 8 waves.
enum Route : int { kRouteShortLo = 0, kRouteShortHi = 1, kRouteLong = 2, kRouteHuge = 3, kNumRoutes = 4 };
constexpr int kShortLoMaxRegion = 2048;   // 64 lanes x 32 columns

constexpr int kMaxCoopWaves = 8;
constexpr int kMaxColsPerLane = 64;
constexpr int kMaxRegion = kMaxCoopWaves * 64 * kMaxColsPerLane;
constexpr int kShortMaxRegion = 64 * kMaxColsPerLane;  // 4096

// Number of LPT buckets per route: cells are bucketed by quarter octaves.
constexpr int kBuckets = 192;

// Layout of the per-stream planning scratch (device memory, int32 words).
struct PlanScratch {
    int32_t *hist;      // [kNumRoutes * kBuckets] histogram, then cursors
    int32_t *counts;    // [kNumRoutes]  pairs per route
    int32_t *queue;     // [kNumRoutes]  persistent work-queue heads
    int32_t *list;      // [kNumRoutes * capacity] pair indices per route
    int64_t capacity;   // pairs the lists can hold
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
};

struct LaunchCfg {
    int short_max;      // r_len <= short_max -> one wave per pair
    int coop_waves;     // waves per workgroup for long pairs
    bool persistent;    // atomic queue + LPT order, device-sized grid
    bool antidiag;      // long pairs on the anti-diagonal LDS kernel
    int short_lo_grid;  // persistent grid sizes (workgroups)
    int short_hi_grid;
    int long_grid;
    int huge_grid;
};

// Planning: route every pair, write sentinel outputs for degenerate and
// invalid pairs, and build per-route lists ordered by decreasing cell count
// (persistent) or in arrival order of the atomics (plain).
hipError_t launch_plan(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg,
                       const PlanScratch &s, hipStream_t stream);
hipError_t launch_short_lo(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg,
                           const PlanScratch &s, hipStream_t stream);
hipError_t launch_short_hi(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg,
                           const PlanScratch &s, hipStream_t stream);
hipError_t launch_long(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg,
                       const PlanScratch &s, hipStream_t stream);
hipError_t launch_huge(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg,
                       const PlanScratch &s, hipStream_t stream);
hipError_t launch_decide(const float *score, int64_t n_pairs, const int64_t *cand_off, const int32_t *cand_cnt,
                         const int32_t *n_events, int64_t n_reads, double b_match, double threshold,
                         int32_t *out_best, double *out_score, uint8_t *out_mapped, hipStream_t stream);

// Occupancy-derived persistent grid sizes (workgroups per CU) for the
// current device.
int short_blocks_per_cu(bool extend, bool hi);
int long_blocks_per_cu(int coop_waves, bool extend, bool antidiag);

}  // namespace ra
