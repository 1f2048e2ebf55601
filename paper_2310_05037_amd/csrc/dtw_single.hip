// dtw_single.hip -- regions of at most kSingleMaxRegion levels: one wave
// sweeps the whole region as a single stripe (see dtw_device.h for the
// layout).
#include "dtw_device.h"

namespace ra {

// At most 32 columns per lane fit 128 VGPRs (4 waves per SIMD), 44 fit 168
// (3 waves), 64 fit 256 (2 waves).
template <int KHI>
constexpr int single_waves() {
    return KHI <= 8 ? 4 : (KHI <= 11 ? 3 : 2);
}

// Two chains per lane (see sweep) for the two-wave kernel of 34..64 columns
// per lane, where fewer waves leave the SIMD fewer independent instructions.
#ifndef RA_SINGLE_HI_ILP2
#define RA_SINGLE_HI_ILP2 0
#endif

// Columns per lane C = 2H for H in [H, HMAX].
template <bool EXT, bool ILP2, int H, int HMAX>
RA_DEV void single_dispatch(int h, const PairView &pv, float &best, int &bj) {
    if constexpr (H <= HMAX) {
        if (h == H) {
            float nc;
            sweep<kSingleColStep * H, EXT, false, false, ILP2>(pv, 0, nullptr, 0.0f, nc, best, bj);
        } else {
            single_dispatch<EXT, ILP2, H + 1, HMAX>(h, pv, best, bj);
        }
    }
}

// Regions of 256(KLO-1)+1 .. 256 KHI levels.
template <bool EXT, int KLO, int KHI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(single_waves<KHI>(), single_waves<KHI>())))
void k_single(PairArrays a, const int32_t *__restrict__ list, const int32_t *__restrict__ count,
              int32_t *queue) {
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
        const int h = (pv.m + 64 * kSingleColStep - 1) / (64 * kSingleColStep);   // C = 2h columns per lane
        float best = __builtin_nanf("");
        int bj = -2;
        single_dispatch<EXT, (KLO > 8 && RA_SINGLE_HI_ILP2 != 0), 4 * (KLO - 1) / kSingleColStep + 1,
                        4 * KHI / kSingleColStep>(h, pv, best, bj);
        if (__lane_id() == 0) {
            a.out_score[p] = best;
            if (a.out_end) a.out_end[p] = bj;
        }
        if (!queue) break;
        int it = 0;
        if (__lane_id() == 0) it = atomicAdd(queue, 1);
        item = __builtin_amdgcn_readfirstlane(it);
    }
}

template <int KLO, int KHI>
static hipError_t launch_single(int route, int pgrid, const PairArrays &a, int64_t n_pairs,
                                const LaunchCfg &cfg, const PlanScratch &s, hipStream_t stream) {
    const int32_t *list = s.list + route * s.capacity;
    const int32_t *count = s.counts + route;
    int32_t *queue = cfg.persistent ? s.queue + route : nullptr;
    // Plain mode: one workgroup per possible item, in list (arrival) order.
    const unsigned grid = cfg.persistent ? (unsigned)pgrid : (unsigned)n_pairs;
    if (a.rows)
        hipLaunchKernelGGL((k_single<true, KLO, KHI>), dim3(grid), dim3(64), 0, stream, a, list, count, queue);
    else
        hipLaunchKernelGGL((k_single<false, KLO, KHI>), dim3(grid), dim3(64), 0, stream, a, list, count, queue);
    return hipGetLastError();
}

hipError_t launch_single_lo(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                            hipStream_t stream) {
    return launch_single<1, 8>(kRouteSingleLo, cfg.lo_grid, a, n_pairs, cfg, s, stream);
}

hipError_t launch_single_hi(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                            hipStream_t stream) {
    return launch_single<9, kSingleHiMaxK>(kRouteSingleHi, cfg.hi_grid, a, n_pairs, cfg, s, stream);
}

template <bool EXT, int KLO, int KHI>
static int blocks_per_cu() {
    int nb = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_single<EXT, KLO, KHI>, 64, 0);
    return nb > 0 ? nb : 1;
}

int single_lo_blocks_per_cu(bool extend) {
    return extend ? blocks_per_cu<true, 1, 8>() : blocks_per_cu<false, 1, 8>();
}

int single_hi_blocks_per_cu(bool extend) {
    return extend ? blocks_per_cu<true, 9, kSingleHiMaxK>() : blocks_per_cu<false, 9, kSingleHiMaxK>();
}

}  // namespace ra
