// dtw_antidiag.hip -- regions longer than 4096 levels in anti-diagonal order.
//
// The paper vectorises its DTW by walking the table anti-diagonal by
// anti-diagonal (Sec. 2.4.4): the cells of one anti-diagonal depend only on
// the two before it, so they can all be computed at once.  This kernel is
// that scheme on one workgroup per pair, kept as the comparison variant of
// the lane-striped kernel (RAWALIGN_LONG_ANTIDIAG):
//   * the query rows are taken in blocks of 256 R (R = 1, 2 or 4 by query
//     length); thread t owns the R consecutive rows i0 + R t .. + R-1, and at
//     step e of the block it computes their cells on anti-diagonal
//     e = (i - i0) + j, so every step is one anti-diagonal of the block;
//   * inside a thread the north, west and north-west neighbours and the
//     levels come from registers (a row's level at step e is the level the
//     row above used at step e-1); only the block-internal boundary crosses
//     threads: thread t writes its last row's value to LDS and thread t+1
//     reads it one step later as the north neighbour of its first row;
//   * the row above the block, D(i0-1, .), comes from the workgroup's row
//     buffer in device memory: the previous block's last row writes it in
//     place as it goes (column j is staged for the new block's first row
//     before its last row rewrites it, at step j + h - 1 >= j); the first
//     block uses row -1 = 0 instead;
//   * the levels and the row above are staged through LDS rings of three
//     chunks of 256 R columns, each loaded one chunk (256 R steps) ahead;
//   * one LDS-only workgroup barrier per step separates the LDS writes of
//     step e from the reads of step e+1 (and the reads of e from the writes
//     of e+1, which reuse the buffer of e-1); a full barrier between blocks
//     makes the row buffer's stores visible.
// Every thread runs the same block and step loops with the same bounds, so
// every thread reaches every barrier.  The thread holding row n-1 tracks the
// running minimum of the last row as the steps pass it (columns increase
// with e, so a strict < keeps the smallest column on ties).
#include "dtw_device.h"

namespace ra {

constexpr int kAdThreads = 256;

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (the prefetches below rely on that).
RA_DEV void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS of one workgroup, sized for the largest R.
constexpr int kAdMaxR = 4;
constexpr int kAdRingMax = 3 * kAdThreads * kAdMaxR;
struct AdShared {
    float edge[2][kAdThreads];     // last row of every thread at steps e-1 / e
    float rring[kAdRingMax];       // levels, chunk k in slot k mod 3
    float uring[kAdRingMax];       // row above the block, same layout
};

// Chunk k = columns [W k, W k + W), W = 256 R, sits in ring slot k mod 3.  At
// step e thread t's first row reads column e - R t in [e - W + R, e], i.e.
// chunks c-1 and c (c = e / W); chunk c+1 is written into the slot of chunk
// c-2 at the last step of chunk c, from registers loaded W steps earlier.
template <int R>
RA_DEV void antidiag_pair(const PairView &pv, float *prow, AdShared &sh, float &best, int &bj) {
    constexpr int W = kAdThreads * R;
    constexpr int RING = 3 * W;
    const int t = threadIdx.x;
    const int n = pv.n;
    const int m = pv.m;
    for (int i0 = 0; i0 < n; i0 += W) {
        const int h = n - i0 < W ? n - i0 : W;   // rows in this block
        const bool first_block = i0 == 0;
        const bool last_block = i0 + h == n;
        const int row0 = R * t;                  // first own row, relative to i0
        // Full barrier: the previous block's row-buffer stores are visible
        // and its last LDS reads are done.
        __syncthreads();
        float qv[R], prev[R], nw[R], rv[R];
#pragma unroll
        for (int s = 0; s < R; ++s) {
            qv[s] = row0 + s < h ? pv.q[i0 + row0 + s] : 0.0f;
            prev[s] = kInf;   // D(i, -1) = +inf until the row's first cell
            nw[s] = kInf;     // D(i-1, -1): +inf (row 0: row -1 is 0 anyway)
            rv[s] = 0.0f;
        }
        float r_nx[R], u_nx[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int c0 = k * kAdThreads + t;          // chunk 0
            const int c1 = W + c0;                      // chunk 1
            sh.rring[c0] = c0 < m ? pv.r[c0] : 0.0f;
            sh.uring[c0] = (!first_block && c0 < m) ? prow[c0] : 0.0f;
            r_nx[k] = c1 < m ? pv.r[c1] : 0.0f;
            u_nx[k] = (!first_block && c1 < m) ? prow[c1] : 0.0f;
        }
        lds_barrier();
        const int n_steps = h + m - 1;
        int ri = (RING - row0) % RING;   // ring index of column e - R t
        int pos = 0;                     // e mod W
        int slot = 1;                    // ring slot of chunk c+1
        int jn = W;                      // first column of the chunk held in r_nx
        for (int e = 0; e < n_steps; ++e) {
            const float *prv = (e & 1) ? sh.edge[0] : sh.edge[1];   // step e-1
            float *cur = (e & 1) ? sh.edge[1] : sh.edge[0];         // step e
            const int j0 = e - row0;                                // column of the first own row
            // Level of the first row from the ring; the others shift down.
#pragma unroll
            for (int s = R - 1; s > 0; --s) rv[s] = rv[s - 1];
            rv[0] = sh.rring[ri];
            // North neighbour of the first row: the row above the block, or
            // the previous thread's last row at step e-1.
            float up = t == 0 ? sh.uring[ri] : prv[t - 1];
#pragma unroll
            for (int s = 0; s < R; ++s) {
                const int j = j0 - s;
                const bool act = row0 + s < h && j >= 0 && j < m;
                const float v = cell(qv[s], rv[s], nw[s], up, prev[s]);
                const float upn = prev[s];   // this row at step e-1: north of row s+1
                if (act) {
                    nw[s] = up;
                    prev[s] = v;
                }
                up = upn;
            }
            // prev[] now holds step e for active rows.
            cur[t] = prev[R - 1];
            // The block's last row: row h-1 = R t_l + s_l.
#pragma unroll
            for (int s = 0; s < R; ++s) {
                const int j = j0 - s;
                if (row0 + s == h - 1 && j >= 0 && j < m) {
                    if (last_block) {
                        if (prev[s] < best) {
                            best = prev[s];
                            bj = j;
                        }
                    } else {
                        prow[j] = prev[s];   // row above the next block (column j was staged long ago)
                    }
                }
            }
            if (pos == W - 1) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    sh.rring[slot * W + k * kAdThreads + t] = r_nx[k];
                    sh.uring[slot * W + k * kAdThreads + t] = u_nx[k];
                }
                jn += W;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int c = jn + k * kAdThreads + t;
                    r_nx[k] = c < m ? pv.r[c] : 0.0f;
                    u_nx[k] = (!first_block && c < m) ? prow[c] : 0.0f;
                }
                slot = slot == 2 ? 0 : slot + 1;
                pos = 0;
            } else {
                ++pos;
            }
            ri = ri == RING - 1 ? 0 : ri + 1;
            lds_barrier();
        }
    }
}

__global__ __launch_bounds__(kAdThreads) void k_antidiag(PairArrays a, const int32_t *__restrict__ list,
                                                         const int32_t *__restrict__ count, int32_t *queue,
                                                         float *rowbuf) {
    __shared__ AdShared sh;
    __shared__ int s_item;
    float *prow = rowbuf + (size_t)blockIdx.x * kMaxRegion;
    const int n_items = *count;
    int item = blockIdx.x;
    for (;;) {
        if (queue) {
            if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
            __syncthreads();
            item = s_item;
            __syncthreads();   // every thread has read s_item before it is written again
        }
        if (item >= n_items) break;   // uniform: item comes from LDS or blockIdx
        const int p = list[item];
        const PairView pv = pair_view<false>(a, p);
        float best = kInf;
        int bj = 0x7fffffff;
        // The planner routes only pairs with 1 <= n <= kEdgeCap and
        // 4096 < m <= kMaxRegion here.  Rows per thread by query length
        // (uniform across the workgroup).
        int R;
        if (pv.n >= 2048)
            R = 4;
        else if (pv.n >= 512)
            R = 2;
        else
            R = 1;
        if (R == 4)
            antidiag_pair<4>(pv, prow, sh, best, bj);
        else if (R == 2)
            antidiag_pair<2>(pv, prow, sh, best, bj);
        else
            antidiag_pair<1>(pv, prow, sh, best, bj);
        // Row n-1 = i0 + R t + s of the last block.
        const int last_rel = (pv.n - 1) % (kAdThreads * R);
        if (threadIdx.x == last_rel / R) {
            a.out_score[p] = best;
            a.out_end[p] = bj;
        }
        if (!queue) item += gridDim.x;
    }
}

hipError_t launch_antidiag(const PairArrays &a, int64_t n_pairs, const LaunchCfg &cfg, const PlanScratch &s,
                           hipStream_t stream) {
    (void)n_pairs;
    if (a.rows || !s.rowbuf) return hipErrorInvalidValue;   // plain batches only (checked on the host before)
    const int32_t *list = s.list + kRouteMulti * s.capacity;
    const int32_t *count = s.counts + kRouteMulti;
    int32_t *queue = cfg.persistent ? s.queue + kRouteMulti : nullptr;
    // One row buffer per workgroup: the grid never exceeds the buffers.
    hipLaunchKernelGGL(k_antidiag, dim3((unsigned)cfg.antidiag_grid), dim3(kAdThreads), 0, stream, a, list, count,
                       queue, s.rowbuf);
    return hipGetLastError();
}

int antidiag_blocks_per_cu() {
    int nb = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_antidiag, kAdThreads, 0);
    return nb > 0 ? nb : 1;
}

}  // namespace ra
