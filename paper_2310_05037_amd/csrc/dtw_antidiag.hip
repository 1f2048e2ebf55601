// dtw_antidiag.hip -- regions above one stripe in anti-diagonal order.
//
// The paper vectorises its DTW by walking the table anti-diagonal by
// anti-diagonal (Sec. 2.4.4): the cells of one anti-diagonal depend only on
// the two before it, so they can all be computed at once.  This kernel is
// that scheme on one workgroup of 256 threads per pair, kept as the
// comparison variant of the lane-striped kernel (RAWALIGN_LONG_ANTIDIAG),
// with the unit of the wavefront widened from one cell to a tile:
//   * the query rows are taken in blocks of 256 R (R = 2 to 8, chosen per
//     pair from a cost model); thread t owns rows R t .. R t + R-1 of every
//     block, and the region's columns are cut into tiles of K = 8;
//   * tiles are numbered in one stream g = rb S + b over (row block rb,
//     column tile b), with a row-block stride S >= the tile count (the tiles
//     b in [tiles, S) are idle).  At step E thread t computes its R x K tile
//     g = E - t, so one step is one anti-diagonal of tiles, and thread 0
//     starts row block rb+1 while the later threads are still in rb: there
//     is no fill or drain between row blocks;
//   * inside a tile the north, west and north-west neighbours come from
//     registers; only tile edges cross threads: thread t writes the K values
//     of its last row to LDS and thread t+1 reads them at the next step as
//     the row above its first row.  Within a wave one buffer suffices (the
//     read of step E+1 follows the write of step E in program order); lane
//     63 hands over to lane 0 of the next wave through a slot
//     double-buffered by step parity.  One LDS barrier per step;
//   * thread 0's row above is the last row of the previous row block, which
//     thread 255 stores into the workgroup's row buffer in device memory S -
//     255 steps before thread 0 needs it; the stride S >= 255 + 4 chunk
//     lengths keeps that store at least one chunk ahead of the staging load
//     that reads it (the first row block uses row -1 = 0);
//   * the levels and thread 0's row above are staged through LDS rings in
//     chunks of 32 tiles (one float per thread), written two chunks ahead of
//     their first use from registers loaded one chunk before that; the query
//     rows of a thread's next row block go to a private LDS slot at such a
//     chunk step, so the step loop never waits for a global load;
//   * rings and edge buffers are split into two halves of four floats per
//     tile, so the 16-byte reads and writes of neighbouring threads fall on
//     consecutive banks.
//   * inside a tile the cells are taken in anti-diagonal order as well, so
//     each cell's min3 -> add pair has independent cells between it and the
//     next use of its result.
// Every thread runs the same step loops with the same bounds, so every
// thread reaches every barrier.  Tiles past the query (rows >= n) are
// computed and discarded, except on the thread t_l that holds row n-1: from
// the step at which it enters the last row block, its rows below n-1 take a
// weight of 0 on the distance term, which turns them into prefix minima of
// row n-1 (the same minimum at the same first column), and it stores the
// last row of each tile into the row buffer.  After the loop the workgroup
// scans that row for its minimum and first column.  Without rows below n-1
// on thread t_l (n-1 is its last row) no step needs the weights.
#include "dtw_device.h"

namespace ra {

constexpr int kAdThreads = 256;
constexpr int kAdK = 8;                                      // columns per tile
constexpr int kAdMaxR = 8;                                   // rows per thread, at most
constexpr int kAdChunk = kAdThreads / kAdK;                  // tiles per staged chunk (32)
constexpr int kAdLvChunks = 10;                              // level ring: 256 / 32 + 2 chunks live
constexpr int kAdUpChunks = 4;                               // row-above ring: >= 3 chunks live
constexpr int kAdLvHalf = 4 * kAdChunk * kAdLvChunks;        // floats per half of the level ring
constexpr int kAdUpHalf = 4 * kAdChunk * kAdUpChunks;
constexpr int kAdMinStride = kAdThreads + 4 * kAdChunk;      // 384 tiles
// Per-step overhead in VALU slots of the cost model: about 28 VALU of edge,
// level and index work per step at R = 8, plus the barrier; 48 picks R best
// on mixed shapes (24 and 96 both measured slower).
constexpr int kAdStepCost = 48;

// LDS layout, in floats.  Every 8-value access (a tile's levels, a row
// segment) is two 16-byte halves at the same offset in half 0 and half 1,
// kAdHalf apart:
//   lv   [kAdLvHalf]   levels of tile g at (4 g) mod kAdLvHalf
//   up   [kAdUpHalf]   thread 0's row above, same layout
//   edge [4 x 256]     last row of thread t at 4 t (read by lane t+1 of the
//                      same wave; single-buffered: within a wave the read of
//                      step E+1 follows the write of step E in program order)
//   bnd  [2 x 4 x 4]   last row of lane 63 of wave w at step parity p, for
//                      lane 0 of wave w+1 (double-buffered across the barrier)
// after both halves, the query rows: thread t's R rows at kAdQ + R t.
constexpr int kAdLv = 0;
constexpr int kAdUp = kAdLv + kAdLvHalf;
constexpr int kAdEdge = kAdUp + kAdUpHalf;
constexpr int kAdBnd = kAdEdge + 4 * kAdThreads;
constexpr int kAdHalf = kAdBnd + 2 * 4 * 4;
constexpr int kAdQ = 2 * kAdHalf;
constexpr int kAdLds = kAdQ + kAdMaxR * kAdThreads;

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (the staging loads rely on that).
RA_DEV void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Per-pair shape of the tile stream (uniform across the workgroup).
struct AdShape {
    int R, W;        // rows per thread, rows per block (256 R)
    int tiles;       // column tiles, ceil(m / K)
    int stride;      // tiles per row block in the stream, max(tiles, kAdMinStride)
    int blocks;      // row blocks, ceil(n / W)
    int last_tile;   // stream index of the last tile with work
    int t_l, s_l;    // thread and row slot of query row n-1
};

RA_DEV AdShape ad_shape(int n, int m, int R) {
    AdShape a;
    a.R = R;
    a.W = kAdThreads * R;
    a.tiles = (m + kAdK - 1) / kAdK;
    a.stride = a.tiles > kAdMinStride ? a.tiles : kAdMinStride;
    a.blocks = (n + a.W - 1) / a.W;
    a.last_tile = (a.blocks - 1) * a.stride + a.tiles - 1;
    const int rel = (n - 1) - (a.blocks - 1) * a.W;
    a.t_l = rel / R;
    a.s_l = rel % R;
    return a;
}

// Steps a shape takes (the last tile reaches thread t_l), times the VALU
// slots of one step.
RA_DEV long long ad_cost(const AdShape &a) {
    return (long long)(a.last_tile + a.t_l + 1) * (3 * a.R * kAdK + kAdStepCost);
}

// One element of a staged chunk: thread u holds column k = u % K of tile
// g = 32 c + u / K.  Levels past the region and idle tiles stage 0; the row
// above is 0 in the first row block (row -1) and read back from the row
// buffer after it.
struct AdStage {
    float lv, up;
};

RA_DEV AdStage ad_stage_load(const PairView &pv, const float *prow, const AdShape &a, int chunk) {
    const int u = threadIdx.x;
    const int g = kAdChunk * chunk + u / kAdK;
    const int rb = g / a.stride;
    const int b = g - rb * a.stride;
    const int col = kAdK * b + u % kAdK;
    const bool in = b < a.tiles && col < pv.m;
    AdStage s;
    s.lv = in ? pv.r[col] : 0.0f;
    s.up = (in && rb >= 1 && rb < a.blocks) ? prow[col] : 0.0f;
    return s;
}

RA_DEV void ad_stage_store(float *f, const AdStage &s, int chunk) {
    const int u = threadIdx.x;
    const int g = kAdChunk * chunk + u / kAdK;
    const int k = u % kAdK;
    float *h = f + (k >> 2) * kAdHalf;
    h[kAdLv + (4 * g + (k & 3)) % kAdLvHalf] = s.lv;
    h[kAdUp + ((4 * g + (k & 3)) & (kAdUpHalf - 1))] = s.up;
}

// Eight values at LDS offset o (half 0) and o + kAdHalf (half 1).
RA_DEV void ld8(const float *f, int o, float (&v)[kAdK]) {
    const float4 a = *reinterpret_cast<const float4 *>(f + o);
    const float4 b = *reinterpret_cast<const float4 *>(f + kAdHalf + o);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

RA_DEV void st8(float *f, int o, const float (&v)[kAdK]) {
    *reinterpret_cast<float4 *>(f + o) = make_float4(v[0], v[1], v[2], v[3]);
    *reinterpret_cast<float4 *>(f + kAdHalf + o) = make_float4(v[4], v[5], v[6], v[7]);
}

// The same at a byte offset (offsets that a step selects per lane).
RA_DEV void ld8b(const float *f, int ob, float (&v)[kAdK]) {
    ld8(reinterpret_cast<const float *>(reinterpret_cast<const char *>(f) + ob), 0, v);
}

RA_DEV void st8b(float *f, int ob, const float (&v)[kAdK]) {
    st8(reinterpret_cast<float *>(reinterpret_cast<char *>(f) + ob), 0, v);
}

// Query rows R t .. R t + R-1 of row block `block` (0 past the query).
template <int R>
RA_DEV void ad_rows_load(const PairView &pv, const AdShape &a, int block, float (&q)[R]) {
#pragma unroll
    for (int s = 0; s < R; ++s) {
        const int i = block * a.W + R * (int)threadIdx.x + s;
        q[s] = i < pv.n ? pv.q[i] : 0.0f;
    }
}

// The cell with a weight on the distance term: c = 1 is the recurrence
// itself (the product is exact, so the fused add rounds as the plain add
// does); c = 0 gives min(NW, N, W), a row that carries the prefix minimum of
// the row above.
RA_DEV float cell_w(float qv, float c, float rv, float diag, float up, float left) {
    return __builtin_fmaf(fabsf(qv - rv), c, fminf(fminf(diag, up), left));
}

// One R x K tile in anti-diagonal order.  above[] holds the row above the
// tile on entry and the tile's last row on exit; left[] the column left of
// the tile on entry and its last column on exit; upleft the north-west
// corner.  The cells (s, k) with s + k = d depend only on diagonals d-1 and
// d-2, so each cell's min3 -> add pair is followed by independent cells of
// the same diagonal instead of waiting on its own result.  WEIGHTED: row s
// takes the weight cv[s] on its distance term.
template <int R, bool WEIGHTED>
RA_DEV void ad_tile(const float (&qv)[R], const float (&cv)[R], const float (&lv)[kAdK], float (&above)[kAdK],
                    float (&left)[R], float upleft) {
    constexpr int K = kAdK;
    float v[R][K];
#pragma unroll
    for (int d = 0; d < R + K - 1; ++d) {
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int k = d - s;
            if (k < 0 || k >= K) continue;
            const float n_ = s == 0 ? above[k] : v[s - 1][k];
            const float w = k == 0 ? left[s] : v[s][k - 1];
            const float nw = s == 0 ? (k == 0 ? upleft : above[k - 1]) : (k == 0 ? left[s - 1] : v[s - 1][k - 1]);
            if constexpr (WEIGHTED)
                v[s][k] = cell_w(qv[s], cv[s], lv[k], nw, n_, w);
            else
                v[s][k] = cell(qv[s], lv[k], nw, n_, w);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) above[k] = v[R - 1][k];
#pragma unroll
    for (int s = 0; s < R; ++s) left[s] = v[s][K - 1];
}

template <int R>
RA_DEV void antidiag_pair(const PairView &pv, float *prow, float *f, const AdShape &a, float &best, int &bj) {
    constexpr int K = kAdK;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int m = pv.m;
    float *qrow = f + kAdQ + R * t;   // this thread's query rows (private slot)
    // Chunks 0 and 1 go straight to the rings; chunk 2 waits in registers.
    ad_stage_store(f, ad_stage_load(pv, prow, a, 0), 0);
    ad_stage_store(f, ad_stage_load(pv, prow, a, 1), 1);
    AdStage staged = ad_stage_load(pv, prow, a, 2);
    // Query rows: block 0 into the private slot now; block B >= 1 is loaded
    // at the first chunk step after thread 255 has taken block B-1's rows
    // and written one chunk step later, before thread 0 starts block B.
    float qst[R];
    ad_rows_load<R>(pv, a, 0, qst);
#pragma unroll
    for (int s = 0; s < R; ++s) qrow[s] = qst[s];
    int q_next = 1;           // next row block whose rows are to be loaded
    bool q_pending = false;   // qst holds rows not yet written to the slot
    float qv[R], left[R];
#pragma unroll
    for (int s = 0; s < R; ++s) {
        qv[s] = 0.0f;
        left[s] = kInf;
    }
    float upleft = kInf;
    // Stream position of this thread's tile: g = E - t, b = column tile
    // within row block rb.  b starts at S - t so that it reaches S (the
    // start of block 0) at g = 0; a step that finds b == S starts a block.
    int rb = -1, b = a.stride - t;
    const int E_end = a.last_tile + a.t_l;   // last step with work (thread t_l, last tile)
    // First step at which thread t_l is in the last row block.  From there
    // on, thread t_l's rows past query row n-1 take weight 0, so the last row
    // of its tiles is row n-1 itself or its prefix minimum (the same minimum
    // at the same first column), and it stores that row into the row buffer
    // (free in the last block: its row above was staged before).
    const int E_track = (a.blocks - 1) * a.stride + a.t_l;
    float cv[R];
#pragma unroll
    for (int s = 0; s < R; ++s) cv[s] = 1.0f;
    // LDS byte offsets of the edge read and write of lanes 1..63 and 0..62
    // (step-independent); lanes 0 and 63 take a wave-uniform slot per step.
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int rd_edge = 4 * (kAdEdge + 4 * (t - 1));
    const int wr_edge = 4 * (kAdEdge + 4 * t);
    float lv[K];   // levels of this step's tile, loaded at the end of the step before
    bool store = false;   // this thread stores its tiles' last row (set at each block start)
    lds_barrier();
    // Level-ring offset of the tile each step loads for the next, tile g + 1
    // (kept in [0, kAdLvHalf) for the negative tiles of the wavefront's
    // arrival).
    int lvi = 4 * (((4 * (1 - t)) % kAdLvHalf + kAdLvHalf) % kAdLvHalf);   // bytes
    ld8(f, kAdLv + ((4 * (-t)) % kAdLvHalf + kAdLvHalf) % kAdLvHalf, lv);
    // One step: this thread's tile g = E - t, the edge handed to thread t+1,
    // the staging of every 32nd step, one barrier.
    auto step = [&](const int E, auto weighted) __attribute__((always_inline)) {
        // Row above the first own row: the left neighbour's last row at
        // step E-1 (lane t-1 of this wave, or lane 63 of the wave before
        // through the boundary slot); for thread 0 the staged row above.
        const int rd0 = 4 * (wv == 0 ? kAdUp + ((4 * E) & (kAdUpHalf - 1)) : kAdBnd + (((E - 1) & 1) * 4 + wv - 1) * 4);
        float above[K];
        ld8b(f, lane == 0 ? rd0 : rd_edge, above);
        const float up_last = above[K - 1];   // north-west of the next tile's first row
        if (b == a.stride) {
            // A new row block: column -1 is +inf, query rows of block rb.
            b = 0;
            ++rb;
#pragma unroll
            for (int s = 0; s < R; ++s) {
                left[s] = kInf;
                qv[s] = qrow[s];
            }
            upleft = kInf;
            store = (t == kAdThreads - 1 && rb < a.blocks - 1) || (t == a.t_l && rb == a.blocks - 1);
        }
        const int g = E - t;
        const bool live = (unsigned)g <= (unsigned)a.last_tile && b < a.tiles;
        if (live) {
            const int j0 = K * b;
            ad_tile<R, decltype(weighted)::value>(qv, cv, lv, above, left, upleft);
            if (store) {
                // Last row of the block (the row above of block rb+1), or
                // thread t_l's last row in the last block.
                if (j0 + K <= m) {
                    *reinterpret_cast<float4 *>(prow + j0) = make_float4(above[0], above[1], above[2], above[3]);
                    *reinterpret_cast<float4 *>(prow + j0 + 4) = make_float4(above[4], above[5], above[6], above[7]);
                } else {
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (j0 + k < m) prow[j0 + k] = above[k];
                }
            }
        }
        upleft = up_last;
        st8b(f, lane == 63 ? 4 * (kAdBnd + ((E & 1) * 4 + wv) * 4) : wr_edge, above);
        // The next step's levels: this barrier's LDS wait covers the load.
        ld8b(f, 4 * kAdLv + lvi, lv);
        lvi = lvi + 16 == 4 * kAdLvHalf ? 0 : lvi + 16;
        if ((E & (kAdChunk - 1)) == kAdChunk - 1) {
            const int c = E / kAdChunk;
            ad_stage_store(f, staged, c + 2);
            staged = ad_stage_load(pv, prow, a, c + 3);
            if (q_pending) {
#pragma unroll
                for (int s = 0; s < R; ++s) qrow[s] = qst[s];
                q_pending = false;
            }
            if (q_next < a.blocks && E >= (q_next - 1) * a.stride + kAdThreads) {
                ad_rows_load<R>(pv, a, q_next, qst);
                q_pending = true;
                ++q_next;
            }
        }
        ++b;
        lds_barrier();
    };
    // Weights are needed only below row n-1 within thread t_l's tile.
    const int E_w = a.s_l == R - 1 ? E_end + 1 : E_track;
    int E = 0;
    for (; E < E_w; ++E) step(E, std::false_type{});
#pragma unroll
    for (int s = 0; s < R; ++s) cv[s] = t == a.t_l && s > a.s_l ? 0.0f : 1.0f;
    for (; E <= E_end; ++E) step(E, std::true_type{});
    // Minimum of the stored row and its first column: a strided scan per
    // thread (four loads in flight; columns increase, so a strict < keeps
    // the first), then across the wave and the four waves.
    __syncthreads();
    float bv = kInf;
    int bc = 0x7fffffff;
    for (int j0 = t; j0 < m; j0 += 4 * kAdThreads) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = j0 + u * kAdThreads < m ? prow[j0 + u * kAdThreads] : kInf;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (v[u] < bv) {
                bv = v[u];
                bc = j0 + u * kAdThreads;
            }
        }
    }
    wave_min(bv, bc);
    float *red = f + kAdEdge;
    if (lane == 0) {
        red[wave] = bv;
        reinterpret_cast<int *>(red)[4 + wave] = bc;
    }
    __syncthreads();
    if (t == 0) {
        best = red[0];
        bj = reinterpret_cast<const int *>(red)[4];
        for (int w = 1; w < kAdThreads / 64; ++w) take_min(best, bj, red[w], reinterpret_cast<const int *>(red)[4 + w]);
    }
}

__global__ __launch_bounds__(kAdThreads) __attribute__((amdgpu_waves_per_eu(5, 5))) void k_antidiag(PairArrays a, const int32_t *__restrict__ list,
                                                         const int32_t *__restrict__ count, int32_t *queue,
                                                         float *rowbuf) {
    __shared__ float4 lds[kAdLds / 4];
    __shared__ int s_item;
    float *f = reinterpret_cast<float *>(lds);
    float *prow = rowbuf + (size_t)blockIdx.x * kMaxRegion;
    const int n_items = *count;
    int item = blockIdx.x;
    for (;;) {
        if (queue) {
            if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
            __syncthreads();
            item = s_item;
        }
        // Every thread has read s_item (before thread 0 writes it again) and
        // finished the previous pair's LDS reads (before the rings are
        // rewritten).
        __syncthreads();
        if (item >= n_items) break;   // uniform: item comes from LDS or blockIdx
        const int p = list[item];
        const PairView pv = pair_view<false>(a, p);
        float best = kInf;
        int bj = 0x7fffffff;
        // The planner routes only pairs with 1 <= n <= kEdgeCap and regions
        // above one stripe here.  Rows per thread: the cheapest R of 2..8
        // under the step-count model (uniform across the workgroup; the
        // largest R on equal cost).
        int R = 8;
        long long cbest = ad_cost(ad_shape(pv.n, pv.m, 8));
        for (int r = 7; r >= 2; --r) {
            const long long c = ad_cost(ad_shape(pv.n, pv.m, r));
            if (c < cbest) {
                cbest = c;
                R = r;
            }
        }
        R = __builtin_amdgcn_readfirstlane(R);
        switch (R) {
        case 8: antidiag_pair<8>(pv, prow, f, ad_shape(pv.n, pv.m, 8), best, bj); break;
        case 7: antidiag_pair<7>(pv, prow, f, ad_shape(pv.n, pv.m, 7), best, bj); break;
        case 6: antidiag_pair<6>(pv, prow, f, ad_shape(pv.n, pv.m, 6), best, bj); break;
        case 5: antidiag_pair<5>(pv, prow, f, ad_shape(pv.n, pv.m, 5), best, bj); break;
        case 4: antidiag_pair<4>(pv, prow, f, ad_shape(pv.n, pv.m, 4), best, bj); break;
        case 3: antidiag_pair<3>(pv, prow, f, ad_shape(pv.n, pv.m, 3), best, bj); break;
        default: antidiag_pair<2>(pv, prow, f, ad_shape(pv.n, pv.m, 2), best, bj); break;
        }
        if (threadIdx.x == 0) {
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
