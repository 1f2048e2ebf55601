// dtw_path.hip -- the warping path of each alignment (RawAlign, arXiv
// 2310.05037, Sec. 2.4: the path can be added to the output).
//
// Given an alignment's start s and end e (the start-of-alignment pass), its
// path is an optimal global path from (0, s) to (n-1, e): global DTW of the
// whole query against r[s..e], entered from the corner D(-1, s-1) = 0.
//
// k_path_dirs: one wave per pair sweeps the n x L table (L = e - s + 1) in
// the lane-striped, skewed order of the other kernels: S stripes of 64 C
// columns (C <= 32), lane k owning C columns of a stripe and computing row
// t - k at step t, the query event and the west value arriving from lane
// k-1 by DPP.  Lane 63 stores the stripe's last column of every row, which
// lane 0 of the next stripe reads back as its west value.  Every cell also
// records which neighbour gave its minimum, north-west before north before
// west on ties, as 2 bits; a lane packs its C codes of a row into one
// 64-bit word, so a row of a stripe is 512 contiguous bytes of the caller's
// workspace.  Per cell: v_sub, v_min3, v_add, two compares and two selects
// for the code, and its insertion into the word.
//
// k_path_trace: one thread per pair follows the codes back from (n-1, L-1)
// to (0, 0) and writes, for every query row i, the region columns lo[i] ..
// hi[i] that the path visits (a monotone path covers a contiguous range of
// every row).
#include "dtw_device.h"
#include "dtw_path.h"

namespace ra {

constexpr int kPathNW = 0, kPathN = 1, kPathW = 2;

template <int C>
RA_DEV void path_pair(const PathArgs &pa, int64_t p, int n, int s, int L, int S) {
    const int lane = opaque_lane();
    const float *rp = pa.r + pa.r_off[p] + s;
    const __amdgpu_buffer_rsrc_t rrs = make_rsrc(rp, L);
    const __amdgpu_buffer_rsrc_t qrs = make_rsrc(pa.q + pa.q_off[p], n);
    uint64_t *base = pa.dirs + pa.dir_off[p];
    // Stripe edge: D(i, last column of the stripe) for every row i.
    float *edge = reinterpret_cast<float *>(base + (int64_t)n * kPathWordsPerRow * S);
    const __amdgpu_buffer_rsrc_t ers = make_rsrc(edge, n);
    const int nm1 = n - 1;
    for (int st = 0; st < S; ++st) {
        const bool ein = st > 0, eout = st + 1 < S;
        const int col0 = st * 64 * C + lane * C;
        float rv[C], A[C];
#pragma unroll
        for (int v = 0; v < C; ++v) {
            const int j = col0 + v;
            const float lv = bload(rrs, j < L ? j : L - 1);
            rv[v] = j < L ? lv : kInf;
            A[v] = kInf;   // row -1: +inf except the corner D(-1, -1) (stripe 0, lane 0)
        }
        uint64_t *dw = base + (int64_t)st * n * kPathWordsPerRow + lane;
        // West value of this step (ecur) and of the previous one (eprev):
        // lane k-1's last column of rows i and i-1; for lane 0 column -1 of
        // the stripe: +inf in the first stripe (whose first previous value is
        // the corner, 0), the previous stripe's edge otherwise (row -1: +inf).
        float ecur = ein ? kInf : 0.0f, eprev, qv = 0.0f;
        float qa = uload(qrs, 0, nm1), qb = uload(qrs, 1, nm1);
        float ea = kInf, eb = kInf;
        if (ein) {
            ea = uload(ers, 0, nm1);
            eb = uload(ers, 1, nm1);
        }
        const int T = n + 63;
        for (int t = 0; t < T; ++t) {
            const float q0 = qa, e0 = ea;
            qa = qb;
            qb = uload(qrs, t + 2, nm1);
            ea = eb;
            if (ein) eb = uload(ers, t + 2, nm1);
            qv = dpp_shr1(q0, qv);
            eprev = ecur;
            ecur = dpp_shr1(ein ? e0 : kInf, A[C - 1]);
            const int i = t - lane;
            const bool valid = (unsigned)i < (unsigned)n;
            float diag = eprev, left = ecur;
            uint64_t code = 0;
#pragma unroll
            for (int v = 0; v < C; ++v) {
                const float up = A[v];
                const float mn = fminf(fminf(diag, up), left);
                const uint32_t c = diag == mn ? kPathNW : (up == mn ? kPathN : kPathW);
                code |= (uint64_t)c << (2 * v);
                const float nv = fabsf(qv - rv[v]) + mn;
                diag = up;
                left = nv;
                A[v] = valid ? nv : A[v];
            }
            if (valid) {
                dw[(int64_t)i * kPathWordsPerRow] = code;
                // Lane 0 read edge[i] two steps before row i; this store
                // (row i, 63 steps later) is for the next stripe.
                if (eout && lane == 63) edge[i] = A[C - 1];
            }
        }
        // Lane 63's edge stores must be visible to lane 0 of the next stripe.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

template <int H>
RA_DEV void path_dispatch(int h, const PathArgs &pa, int64_t p, int n, int s, int L, int S) {
    if constexpr (H <= kPathStripeCols / 128) {
        if (h == H)
            path_pair<2 * H>(pa, p, n, s, L, S);
        else
            path_dispatch<H + 1>(h, pa, p, n, s, L, S);
    }
}

// Stripes of a pair's interval: S stripes of 64 C columns, C = 2h.
RA_DEV void path_shape(int L, int &S, int &h) {
    S = (L + kPathStripeCols - 1) / kPathStripeCols;
    h = (L + 128 * S - 1) / (128 * S);
}

// Interval of pair p, or a sentinel: -1 / -2 from the start pass (empty
// query or region / invalid slice), -4 when the pair's workspace range is
// missing or too small.
RA_DEV int path_interval(const PathArgs &pa, int64_t p, int &n, int &s, int &L) {
    n = pa.q_len[p];
    const int e = pa.end[p];
    s = pa.start[p];
    if (e < 0) return e;
    const int m = pa.r_len[p];
    const int64_t qo = pa.q_off[p], ro = pa.r_off[p];
    if (n < 1 || s < 0 || s > e || e >= m || qo < 0 || ro < 0 || qo + n > pa.q_size || ro + m > pa.r_size)
        return -2;
    L = e - s + 1;
    const int64_t off = pa.dir_off[p];
    if (off < 0 || off > pa.dir_size || path_words(n, L) > pa.dir_size - off) return -4;
    return 0;
}

__global__ __launch_bounds__(64) void k_path_dirs(PathArgs pa) {
    const int64_t p = blockIdx.x;
    int n = 0, s = 0, L = 0;
    if (path_interval(pa, p, n, s, L) != 0) return;
    int S, h;
    path_shape(L, S, h);
    path_dispatch<1>(h, pa, p, n, s, L, S);
}

__global__ void k_path_trace(PathArgs pa) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= pa.n_pairs) return;
    int n = 0, s = 0, L = 0;
    const int st = path_interval(pa, p, n, s, L);
    const int64_t off = pa.path_off[p];
    const int rows = pa.q_len[p];
    if (rows <= 0 || off < 0 || off > pa.path_size || rows > pa.path_size - off) return;
    int32_t *lo = pa.path_lo + off;
    int32_t *hi = pa.path_hi + off;
    if (st != 0) {
        for (int i = 0; i < rows; ++i) lo[i] = hi[i] = st;
        return;
    }
    int S, h;
    path_shape(L, S, h);
    const int C = 2 * h, Wst = 64 * C;
    const uint64_t *base = pa.dirs + pa.dir_off[p];
    int i = n - 1, j = L - 1;
    hi[i] = s + j;
    // Column j as (stripe sj, lane li, bit pair v), stepped down with j.
    int sj = j / Wst, li = (j - sj * Wst) / C, v = (j - sj * Wst) - li * C;
    // The word of the current cell is kept while west moves stay inside it.
    int64_t widx = -1;
    uint64_t w = 0;
    // Every step lowers i + j; the edges of the table allow only one move
    // (west along row 0, north along column 0), whatever the codes say.
    for (;;) {
        lo[i] = s + j;
        if (i == 0 && j == 0) break;
        const int64_t k = ((int64_t)sj * n + i) * kPathWordsPerRow + li;
        if (k != widx) {
            widx = k;
            w = base[k];
        }
        int d = (int)((w >> (2 * v)) & 3);
        if (i == 0) d = kPathW;
        else if (j == 0) d = kPathN;
        if (d != kPathN) {   // west or north-west: one column left
            --j;
            if (--v < 0) {
                v = C - 1;
                if (--li < 0) {
                    li = 63;
                    --sj;
                }
            }
        }
        if (d != kPathW) {   // north or north-west: one row up
            --i;
            hi[i] = s + j;
        }
    }
}

hipError_t launch_path(const PathArgs &pa, hipStream_t stream) {
    if (pa.n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_path_dirs, dim3((unsigned)pa.n_pairs), dim3(64), 0, stream, pa);
    hipLaunchKernelGGL(k_path_trace, dim3((unsigned)((pa.n_pairs + 63) / 64)), dim3(64), 0, stream, pa);
    return hipGetLastError();
}

}  // namespace ra
