// dtw_multi.hip -- regions longer than 4096 levels: one wave sweeps S column
// stripes one after another.  Lane 63 writes each stripe's last column to
// the wave's own edge slot in device memory; the next stripe's lane 0 reads
// it back as its left neighbour.  Waves never wait for each other.
#include "dtw_device.h"

namespace ra {

template <int C, bool EXT>
RA_DEV void multi_pair(const PairView &pv, int S, float *edge, float &best, int &bj) {
    best = kInf;
    bj = 0x7fffffff;
    float corner = 0.0f;   // D(-1, col_base-1) of the next stripe
    for (int s = 0; s < S; ++s) {
        float b, nc;
        int j;
        if (s == 0)
            sweep<C, EXT, false, true, true>(pv, 0, edge, 0.0f, nc, b, j);
        else
            sweep<C, EXT, true, true, true>(pv, s * 64 * C, edge, corner, nc, b, j);
        corner = nc;
        take_min(best, bj, b, j);
        // Lane 63's edge stores must be visible to lane 0 of the next stripe.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// Columns per lane C = 4k, k in 9..16 for every multi-stripe region.
template <bool EXT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2)))
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
        int S, k;
        stripe_shape(pv.m, S, k);
        float best = __builtin_nanf("");
        int bj = -2;
#define RA_CASE(K) \
    if (k == K) multi_pair<4 * K, EXT>(pv, S, edge, best, bj);
        RA_CASE(9) RA_CASE(10) RA_CASE(11) RA_CASE(12) RA_CASE(13) RA_CASE(14) RA_CASE(15) RA_CASE(16)
#undef RA_CASE
        if (__lane_id() == 0) {
            a.out_score[p] = best;
            a.out_end[p] = bj;
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
