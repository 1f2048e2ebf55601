// dtw_multi.hip -- regions longer than 4096 levels: one wave sweeps S column
// stripes of at most 256 kMultiMaxK columns (2048 by default) one after
// another.  Lane 63 writes each stripe's last column to the wave's own edge
// slot in device memory; the next stripe's lane 0 reads it back as its left
// neighbour.  Waves never wait for each other.
#include "dtw_device.h"

namespace ra {

// Waves per SIMD the register budget of the widest stripe allows.
#ifdef RA_MULTI_WAVES
constexpr int kMultiWaves = RA_MULTI_WAVES;
#else
constexpr int kMultiWaves = kMultiMaxK <= 8 ? 4 : (kMultiMaxK <= 12 ? 3 : 2);
#endif

// Columns per lane C = 2H for every H in [kMultiMinH, kMultiMaxH].
template <int H, bool EXT>
RA_DEV void multi_dispatch(int h, const PairView &pv, int S, float *edge, float &best, int &bj) {
    if constexpr (H <= kMultiMaxH) {
        if (h == H)
            multi_pair<kMultiColStep * H, EXT>(pv, S, edge, best, bj);
        else
            multi_dispatch<H + 1, EXT>(h, pv, S, edge, best, bj);
    }
}

template <bool EXT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kMultiWaves, kMultiWaves)))
void k_multi(PairArrays a, const int32_t *__restrict__ list, const int32_t *__restrict__ count,
             int32_t *queue, float *edge_base) {
    float *edge = edge_base + (size_t)blockIdx.x * kEdgeCap;
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
        int S, h;
        stripe_shape(pv.m, S, h, false);
        float best = __builtin_nanf("");
        int bj = -2;
        multi_dispatch<kMultiMinH, EXT>(h, pv, S, edge, best, bj);
        if (__lane_id() == 0) {
            a.out_score[p] = best;
            if (a.out_end) a.out_end[p] = bj;
        }
        if (queue) {
            int it = 0;
            if (__lane_id() == 0) it = atomicAdd(queue, 1);
            item = __builtin_amdgcn_readfirstlane(it);
        } else {
            item += gridDim.x;   // plain mode: static round robin in arrival order
        }
    }
}

hipError_t launch_multi(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                        hipStream_t stream) {
    (void)n_pairs;
    const int32_t *list = s.list + kRouteMulti * s.capacity;
    const int32_t *count = s.counts + kRouteMulti;
    int32_t *queue = cfg.persistent ? s.queue + kRouteMulti : nullptr;
    // One edge slot per workgroup: the grid never exceeds the slots.
    const unsigned grid = (unsigned)cfg.multi_grid;
    if (a.rows)
        hipLaunchKernelGGL(k_multi<true>, dim3(grid), dim3(64), 0, stream, a, list, count, queue, s.edge);
    else
        hipLaunchKernelGGL(k_multi<false>, dim3(grid), dim3(64), 0, stream, a, list, count, queue, s.edge);
    return hipGetLastError();
}

int multi_blocks_per_cu(bool extend) {
    int nb = 0;
    if (extend)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_multi<true>, 64, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_multi<false>, 64, 0);
    return nb > 0 ? nb : 1;
}

}  // namespace ra
