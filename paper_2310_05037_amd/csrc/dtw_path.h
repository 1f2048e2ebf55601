// dtw_path.h -- warping path of an alignment (kernels in dtw_path.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ra {

// Widest stripe of the direction pass: 64 lanes x 32 columns.
constexpr int kPathStripeCols = 64 * 32;
// Direction words per query row and stripe: one 64-bit word (2 bits per
// column, up to 32 columns) per lane.
constexpr int kPathWordsPerRow = 64;

// Workspace words pair p needs for an interval of L levels: per stripe and
// row one word per lane, plus one word per row for the stripe edge.
__host__ __device__ inline int64_t path_words(int64_t n, int64_t L) {
    const int64_t S = (L + kPathStripeCols - 1) / kPathStripeCols;
    return n * (kPathWordsPerRow * S + 1);
}

struct PathArgs {
    const float *q;
    int64_t q_size;
    const int64_t *q_off;
    const int32_t *q_len;
    const float *r;
    int64_t r_size;
    const int64_t *r_off;
    const int32_t *r_len;
    const int32_t *start;   // per pair, from the start-of-alignment pass
    const int32_t *end;
    int64_t n_pairs;
    const int64_t *dir_off;   // per pair: first workspace word
    uint64_t *dirs;           // caller's workspace
    int64_t dir_size;         // words
    const int64_t *path_off;
    int32_t *path_lo;
    int32_t *path_hi;
    int64_t path_size;
};

hipError_t launch_path(const PathArgs &pa, hipStream_t stream);

}  // namespace ra
