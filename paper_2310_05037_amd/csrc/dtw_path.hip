// dtw_path.hip -- the warping path of each alignment (RawAlign, arXiv
// 2310.05037, Sec. 2.4: the path can be added to the output).
//
// Given an alignment's start s and end e (the start-of-alignment pass), its
// path is an optimal global path from (0, s) to (n-1, e): global DTW of the
// whole query against r[s..e], entered from the corner D(-1, s-1) = 0.
//
// k_path_dirs: one wave per pair sweeps the n x L table (L = e - s + 1 <=
// 2048) in the lane-striped, skewed order of the other kernels (lane k owns
// columns [kC, kC + C), computes row t - k at step t; the query event and
// the west value arrive from lane k-1 by DPP).  Every cell also records
// which neighbour gave its minimum, north-west before north before west on
// ties, as 2 bits; a lane packs its C codes of a row into one 64-bit word,
// so a row of the wave is 512 contiguous bytes.  Per cell: v_sub, v_min3,
// v_add, two compares and two selects for the code, and its shift into the
// word.
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
RA_DEV void path_pair(const PathArgs &pa, int64_t p, int n, int s, int L) {
    const int lane = opaque_lane();
    const int col0 = lane * C;
    const float *rp = pa.r + pa.r_off[p] + s;
    const __amdgpu_buffer_rsrc_t rrs = make_rsrc(rp, L);
    const __amdgpu_buffer_rsrc_t qrs = make_rsrc(pa.q + pa.q_off[p], n);
    float rv[C], A[C];
#pragma unroll
    for (int v = 0; v < C; ++v) {
        const int j = col0 + v;
        const float lv = bload(rrs, j < L ? j : L - 1);
        rv[v] = j < L ? lv : kInf;
        A[v] = kInf;   // row -1: +inf except the corner, which enters through lane 0
    }
    uint64_t *dw = pa.dirs + (size_t)p * pa.max_query * kPathWordsPerRow + lane;
    // West value of this step (ecur) and of the previous one (eprev): lane
    // k-1's last column of rows i and i-1.  Lane 0 holds +inf (column -1),
    // except that its first previous value is the corner D(-1, -1) = 0.
    float ecur = 0.0f, eprev, qv = 0.0f;
    const int nm1 = n - 1;
    float qa = uload(qrs, 0, nm1), qb = uload(qrs, 1, nm1);
    const int T = n + 63;
    for (int t = 0; t < T; ++t) {
        const float q0 = qa;
        qa = qb;
        qb = uload(qrs, t + 2, nm1);
        qv = dpp_shr1(q0, qv);
        eprev = ecur;
        ecur = dpp_shr1(kInf, A[C - 1]);
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
        if (valid) dw[(size_t)i * kPathWordsPerRow] = code;
    }
}

template <int H>
RA_DEV void path_dispatch(int h, const PathArgs &pa, int64_t p, int n, int s, int L) {
    if constexpr (H <= kPathMaxCols / 128) {
        if (h == H)
            path_pair<2 * H>(pa, p, n, s, L);
        else
            path_dispatch<H + 1>(h, pa, p, n, s, L);
    }
}

// Interval of pair p, or a sentinel: -1 / -2 from the start pass (empty
// query or region / invalid slice), -4 when the path is not recorded (more
// than max_query events, or an interval wider than kPathMaxCols levels).
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
    if (n > pa.max_query || L > kPathMaxCols) return -4;
    return 0;
}

__global__ __launch_bounds__(64) void k_path_dirs(PathArgs pa) {
    const int64_t p = blockIdx.x;
    int n = 0, s = 0, L = 0;
    if (path_interval(pa, p, n, s, L) != 0) return;
    path_dispatch<1>((L + 127) / 128, pa, p, n, s, L);
}

__global__ void k_path_trace(PathArgs pa) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= pa.n_pairs) return;
    int n = 0, s = 0, L = 0;
    const int st = path_interval(pa, p, n, s, L);
    const int64_t off = pa.path_off[p];
    const int rows = pa.q_len[p];
    if (rows <= 0 || off < 0 || off + rows > pa.path_size) return;
    int32_t *lo = pa.path_lo + off;
    int32_t *hi = pa.path_hi + off;
    if (st != 0) {
        for (int i = 0; i < rows; ++i) lo[i] = hi[i] = st;
        return;
    }
    const int C = 2 * ((L + 127) / 128);
    const uint64_t *dw = pa.dirs + (size_t)p * pa.max_query * kPathWordsPerRow;
    int i = n - 1, j = L - 1;
    hi[i] = s + j;
    // Every step lowers i + j; the edges of the table allow only one move
    // (west along row 0, north along column 0), whatever the codes say.
    for (;;) {
        lo[i] = s + j;
        if (i == 0 && j == 0) break;
        int d = (int)((dw[(size_t)i * kPathWordsPerRow + j / C] >> (2 * (j % C))) & 3);
        if (i == 0) d = kPathW;
        else if (j == 0) d = kPathN;
        if (d == kPathW) {
            --j;
        } else {
            if (d == kPathNW) --j;
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
