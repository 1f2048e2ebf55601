// dtw_path.h -- warping path of an alignment (kernels in dtw_path.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ra {

// Widest interval [start, end] whose path is recorded: 64 lanes x 32 columns.
constexpr int kPathMaxCols = 64 * 32;
// Direction words per recorded query row: one 64-bit word (2 bits per
// column, up to 32 columns) per lane.
constexpr int kPathWordsPerRow = 64;

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
    int max_query;          // rows of direction words per pair
    uint64_t *dirs;         // [n_pairs][max_query][kPathWordsPerRow]
    const int64_t *path_off;
    int32_t *path_lo;
    int32_t *path_hi;
    int64_t path_size;
};

hipError_t launch_path(const PathArgs &pa, hipStream_t stream);

}  // namespace ra
