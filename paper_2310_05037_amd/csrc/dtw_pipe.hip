// dtw_pipe.hip -- regions longer than one stripe on W cooperating waves.
//
// The single-wave multi-stripe kernel (dtw_multi.hip) sweeps a pair's S
// stripes one after another, so a pair costs S * (n + 64) steps of one wave,
// and a batch with fewer pairs than SIMDs leaves most of the chip idle (the
// 1,024-pair long-problem stress holds one wave per SIMD).  Here the W waves
// of a workgroup share each pair: wave w sweeps stripes w, w + W, w + 2W, ...
// with the same lane-striped sweep, and stripe s starts as soon as stripe
// s - 1 has stored the edge rows it needs, so the stripes of a pair run
// concurrently, each one block of rows behind its left neighbour.
//
// Hand-over, without workgroup barriers:
//   * edges: lane 63 of stripe s stores its last column, one value per row,
//     into the workgroup's edge column in device memory, in place: row i is
//     written by stripe s - 1, read by stripe s, then rewritten by stripe s,
//     always in that order because stripe s reads row i only after stripe
//     s - 1 published it and rewrites it only after reading it;
//   * progress: every block of steps a stripe publishes how many edge rows
//     it has stored (release, then an LDS store), and a stripe about to load
//     edge rows waits until its left neighbour has published them (LDS load,
//     then acquire);
//   * the pair: the wave that finishes a pair last combines the waves'
//     minima, writes the result, clears the counters, takes the next pair
//     from the queue and releases it through an epoch counter in LDS; the
//     other waves wait on that counter.  The pair index reaches every wave
//     through readfirstlane, so all per-pair control flow is scalar.
// Every wait is a spin on an LDS counter capped at kPipeSpinTicks of the
// constant 100 MHz clock (far beyond any legal wait); a wait that times out
// marks the pair failed, its result becomes NaN with end -5, and every wave
// still runs to the end of its work, so the kernel always terminates.  The
// one workgroup barrier is at entry, before any branch, to initialise LDS.
#include "dtw_device.h"

namespace ra {

// Steps between progress publications.  A stripe can start once its left
// neighbour has published a block of rows past the 64-step skew, so each
// stripe trails the one before by about 64 + 2 blocks of rows.  The
// streaming extension sweeps 400-row chunks, where that lag over up to 8
// stripes is most of a chunk's sweep: it publishes every 8 steps.  Plain
// batches sweep whole queries of thousands of rows and keep 64, where each
// publication's fence and spin cost more than the shorter lag saves.
template <bool EXT>
constexpr int pipe_block() { return EXT ? 8 : 64; }
constexpr uint64_t kPipeSpinTicks = 500000000ull;   // 5 s
constexpr int kPipeMaxStripes = kMaxRegion / 2048;   // 32: stripes are at most 2048 columns wide
static_assert(256 * kMultiMaxK <= 2048, "the pipeline's stripe arrays assume stripes of at most 2048 columns");
constexpr int kPipeWavesPerSimd = 4;

struct PipeShared {
    int32_t epoch;                        // pairs released to the workgroup
    int32_t item;                         // list index of the current pair
    int32_t finished;                     // waves done with the current pair
    int32_t failed;                       // a wait of the current pair timed out
    int32_t progress[kPipeMaxStripes];    // edge rows of stripe s stored and published
    float corner[kPipeMaxStripes + 1];    // row -1 left of stripe s (D(-1, col_base - 1))
    float part_v[kPipeMaxWaves];          // each wave's minimum over its stripes
    int32_t part_j[kPipeMaxWaves];
};

RA_DEV int lds_load(int32_t *p) {
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
}

RA_DEV void lds_store(int32_t *p, int v) {
    if (__lane_id() == 0) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

RA_DEV uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// Spin until *p >= target; false after the time cap.
RA_DEV bool spin_until(int32_t *p, int target) {
    const uint64_t deadline = now_ticks() + kPipeSpinTicks;
    for (;;) {
        if (lds_load(p) >= target) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            return true;
        }
        if (now_ticks() > deadline) return false;
        __builtin_amdgcn_s_sleep(2);
    }
}

template <int B>
struct PipeSync {
    static constexpr bool kActive = true;
    static constexpr int kBlock = B;
    PipeShared *sh;
    int s;   // this stripe

    RA_DEV bool wait(int rows) {
        if (lds_load(&sh->failed)) return false;
        if (spin_until(&sh->progress[s - 1], rows)) return true;
        lds_store(&sh->failed, 1);
        return false;
    }
    RA_DEV void publish(int rows) {
        // lane 63's edge stores (and the corner below) before the count
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        lds_store(&sh->progress[s], rows);
    }
    RA_DEV void set_corner(float v) {
        if (__lane_id() == 0) sh->corner[s + 1] = v;
    }
    RA_DEV float corner() { return sh->corner[s]; }
};

template <int C, bool EXT>
RA_DEV void pipe_stripe(const PairView &pv, int s, float *edge, PipeShared *sh, float &b, int &j) {
    using Sync = PipeSync<pipe_block<EXT>()>;
    Sync sync{sh, s};
    float nc;
    if (s == 0)
        sweep<C, EXT, false, true, false, Sync>(pv, 0, edge, 0.0f, nc, b, j, &sync);
    else
        sweep<C, EXT, true, true, false, Sync>(pv, s * 64 * C, edge, 0.0f, nc, b, j, &sync);
}

// Columns per lane C = step * H for every H the multi-stripe shapes use.
template <int H, bool EXT>
RA_DEV void pipe_dispatch(int h, const PairView &pv, int s, float *edge, PipeShared *sh, float &b, int &j) {
    if constexpr (H <= kMultiMaxH) {
        if (h == H)
            pipe_stripe<kMultiColStep * H, EXT>(pv, s, edge, sh, b, j);
        else
            pipe_dispatch<H + 1, EXT>(h, pv, s, edge, sh, b, j);
    }
}

template <bool EXT, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(kPipeWavesPerSimd, kPipeWavesPerSimd)))
void k_pipe(PairArrays a, const int32_t *__restrict__ list, const int32_t *__restrict__ count, int32_t *queue,
            float *edge_base) {
    __shared__ PipeShared sh;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = __lane_id();
    float *edge = edge_base + (size_t)blockIdx.x * kEdgeCap;
    const int n_items = *count;
    for (int i = threadIdx.x; i < kPipeMaxStripes; i += blockDim.x) sh.progress[i] = 0;
    if (threadIdx.x == 0) {
        sh.finished = 0;
        sh.failed = 0;
        sh.item = queue ? atomicAdd(queue, 1) : (int)blockIdx.x;
        sh.epoch = 1;
    }
    __syncthreads();   // the only workgroup barrier: LDS initialised, first pair released
    int seen = 0;
    for (;;) {
        if (!spin_until(&sh.epoch, seen + 1)) break;
        ++seen;
        const int item = lds_load(&sh.item);
        if (item >= n_items) break;
        const int p = list[item];
        // Forward subsequence alignments only (the boundary and direction
        // flags are compile-time false here, which keeps the sweep within
        // its register budget); the ABI sends global and reversed passes to
        // the single-wave kernel.
        PairView pv = pair_view<EXT>(a, p);
        pv.corner = false;
        pv.fixed_end = false;
        pv.reverse = false;
        int S, h;
        stripe_shape(pv.m, S, h, false);
        // Balance: round the stripe count up to a multiple of W (narrower
        // stripes, every wave the same number) when those stripes still have
        // an instantiated width and all start inside the region.  Results do
        // not depend on the stripe layout.
        {
            constexpr int group = 64 * kMultiColStep;
            const int Sb = (S + W - 1) / W * W;
            const int hb = (pv.m + group * Sb - 1) / (group * Sb);
            if (Sb <= kPipeMaxStripes && hb >= kMultiMinH && group * hb * (Sb - 1) < pv.m) {
                S = Sb;
                h = hb;
            }
        }
        float best = kInf;
        int bj = 0x7fffffff;
        for (int s = wave; s < S; s += W) {
            float b;
            int j;
            pipe_dispatch<kMultiMinH, EXT>(h, pv, s, edge, &sh, b, j);
            take_min(best, bj, b, j);
        }
        if (lane == 0) {
            sh.part_v[wave] = best;
            sh.part_j[wave] = bj;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        int old = 0;
        if (lane == 0) old = __hip_atomic_fetch_add(&sh.finished, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        old = __builtin_amdgcn_readfirstlane(old);
        if (old == W - 1) {
            // The last wave of this pair: every other wave has stored its
            // minimum and left the pair's stripes.
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            float v = sh.part_v[0];
            int jj = sh.part_j[0];
            for (int w = 1; w < W; ++w) take_min(v, jj, sh.part_v[w], sh.part_j[w]);
            const bool failed = lds_load(&sh.failed) != 0;
            if (lane == 0) {
                a.out_score[p] = failed ? __builtin_nanf("") : v;
                if (a.out_end) a.out_end[p] = failed ? -5 : jj;
            }
            for (int i = lane; i < kPipeMaxStripes; i += 64) sh.progress[i] = 0;
            lds_store(&sh.finished, 0);
            lds_store(&sh.failed, 0);
            int next = 0;
            // persistent: the queue; plain: static round robin in arrival order
            if (lane == 0) next = queue ? atomicAdd(queue, 1) : item + (int)gridDim.x;
            lds_store(&sh.item, __builtin_amdgcn_readfirstlane(next));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            lds_store(&sh.epoch, seen + 1);
        }
    }
}

template <int W>
static hipError_t launch_pipe_w(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                                hipStream_t stream) {
    const int32_t *list = s.list + kRouteMulti * s.capacity;
    const int32_t *count = s.counts + kRouteMulti;
    int32_t *queue = cfg.persistent ? s.queue + kRouteMulti : nullptr;
    // One edge column per workgroup: the grid never exceeds the slots.
    (void)n_pairs;
    const unsigned grid = (unsigned)cfg.multi_grid;
    if (a.rows)
        hipLaunchKernelGGL((k_pipe<true, W>), dim3(grid), dim3(64 * W), 0, stream, a, list, count, queue, s.edge);
    else
        hipLaunchKernelGGL((k_pipe<false, W>), dim3(grid), dim3(64 * W), 0, stream, a, list, count, queue, s.edge);
    return hipGetLastError();
}

hipError_t launch_pipe(int waves, const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                       hipStream_t stream) {
    switch (waves) {
        case 2: return launch_pipe_w<2>(a, n_pairs, cfg, s, stream);
        case 4: return launch_pipe_w<4>(a, n_pairs, cfg, s, stream);
        case 8: return launch_pipe_w<8>(a, n_pairs, cfg, s, stream);
        default: return hipErrorInvalidValue;
    }
}

template <int W>
static int pipe_blocks_w(bool extend) {
    int nb = 0;
    if (extend)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pipe<true, W>, 64 * W, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pipe<false, W>, 64 * W, 0);
    return nb > 0 ? nb : 1;
}

int pipe_blocks_per_cu(int waves, bool extend) {
    switch (waves) {
        case 2: return pipe_blocks_w<2>(extend);
        case 4: return pipe_blocks_w<4>(extend);
        case 8: return pipe_blocks_w<8>(extend);
        default: return 1;
    }
}

}  // namespace ra
