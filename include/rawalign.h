/*
 * rawalign.h -- C ABI of librawalign.so, batched subsequence dynamic time
 * warping (DTW) for raw nanopore signal alignment on AMD MI355X (gfx950).
 *
 * Method: RawAlign (arXiv 2310.05037).  The alignment step (Sec. 2.1.3)
 * re-evaluates every candidate region left by chaining with DTW (Sec. 2.2):
 * a table whose cells add the numerical difference of a read event and a
 * reference level (no fixed indel penalty) to the smallest of the north,
 * north-west and west neighbours.  The read is aligned whole against a region
 * that is longer than it, so the path may start and end anywhere in the
 * region (subsequence DTW):
 *
 *   c(i,j)  = |q_i - r_j|,        D(-1,j) = 0 (j >= -1),  D(i,-1) = +inf,
 *   D(i,j)  = c(i,j) + min{ D(i-1,j-1), D(i-1,j), D(i,j-1) },
 *   C_DTW   = min_j D(n-1,j),     end = smallest j attaining C_DTW.
 *
 * All arithmetic is IEEE float32; every cell is one rounded subtraction, an
 * exact |.|, an exact min and one rounded addition, so results do not depend
 * on the order in which cells are evaluated (every kernel variant and every
 * launch configuration returns bit-identical scores and ends).
 *
 * Conventions shared by all entry points
 *  - Pointers documented as "device" must point to device memory (hipMalloc,
 *    torch CUDA tensors); "host" pointers to host memory.  The caller owns all
 *    memory passed in; the library never frees it.  Inputs must stay valid
 *    and unmodified until the stream reaches the call.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *    enqueued asynchronously on it; the host never reads device data, so a
 *    call returns before the GPU has finished.
 *  - Pair layout: pair p aligns q[q_off[p] .. q_off[p]+q_len[p]) against
 *    r[r_off[p] .. r_off[p]+r_len[p]).  Offsets are in elements.  Pairs may
 *    share query slices (one read, many candidates) and region slices may
 *    alias one reference-level array; nothing is copied.
 *  - Return value: RAWALIGN_OK (0) or a negative error code; the message of
 *    the last error on the calling thread is rawalign_last_error().  Argument
 *    errors are detected on the host before anything is enqueued.
 *  - Per-pair conditions that only the device can see (it alone reads the
 *    offset and length arrays) give sentinel outputs, never faults:
 *      q_len == 0                   -> score 0,    end -1
 *      r_len == 0 (and q_len > 0)   -> score +inf, end -1
 *      negative length, or a slice outside [0, q_size) / [0, r_size),
 *      or r_len > RAWALIGN_MAX_REGION, or q_len > RAWALIGN_MAX_QUERY
 *                                     -> score NaN, end -2 (pair skipped)
 */
#ifndef RAWALIGN_H
#define RAWALIGN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RAWALIGN_OK 0
#define RAWALIGN_EINVAL (-1)      /* bad argument (null pointer, negative count, bad option) */
#define RAWALIGN_EHIP (-2)        /* HIP runtime or launch error; message keeps hipGetErrorString */
#define RAWALIGN_ENOMEM (-3)      /* internal scratch allocation failed */
#define RAWALIGN_ENODEV (-4)      /* no usable gfx950 device */

/* Longest region (levels) a pair may have: 16 stripes of 64 lanes x 64
 * columns per lane. */
#define RAWALIGN_MAX_REGION 65536
/* Longest query (events) a pair may have; a pair whose region is longer
 * than one stripe (4096 levels) may have at most RAWALIGN_MAX_QUERY_LONG. */
#define RAWALIGN_MAX_QUERY (1 << 28)
#define RAWALIGN_MAX_QUERY_LONG 16384

/* Scheduling modes of rawalign_dtw_batch_ex. */
#define RAWALIGN_MODE_PLAIN 0       /* one workgroup per pair in arrival order, fixed grids */
#define RAWALIGN_MODE_PERSISTENT 1  /* device-sized grids, atomic work queues, longest pairs first */

/* Kernels for regions longer than one stripe (above opts.single_max levels). */
#define RAWALIGN_LONG_STRIPED 0     /* one wave sweeps the stripes in turn, edges through device memory */
#define RAWALIGN_LONG_ANTIDIAG 1    /* one 256-thread workgroup per pair sweeps anti-diagonals of R x 8 tiles,
                                       edges through LDS (Sec. 2.4.4);
                                       plain batches only (rawalign_dtw_extend rejects it) */
#define RAWALIGN_LONG_PIPELINE 2    /* opts.pipe_waves waves share each pair, one stripe each in turn, the
                                       stripes pipelined: a stripe starts as soon as its left neighbour has
                                       stored the edge rows it needs (waits on LDS counters, no barriers) */

/* opts.flags */
#define RAWALIGN_FLAG_TIMING 1      /* record hipEvents around every kernel (rawalign_last_timing) */
#define RAWALIGN_FLAG_SPAN_GIVEN 2  /* rawalign_dtw_path only: out_score, out_end and out_start already hold
                                       rawalign_dtw_span's result for these pairs; its two passes are skipped
                                       (a caller that sized the direction workspace from those intervals) */

typedef struct rawalign_opts {
    int32_t mode;               /* RAWALIGN_MODE_* */
    int32_t long_kernel;        /* RAWALIGN_LONG_* */
    int32_t lo_waves_per_cu;    /* persistent grid of the <= 2048-level kernel, per CU (0 = occupancy limit) */
    int32_t hi_waves_per_cu;    /* same, 2049..4096 levels */
    int32_t long_waves_per_cu;  /* same, > 4096 levels (anti-diagonal kernel: workgroups per CU, 0 = occupancy, 5) */
    int32_t streams;            /* 1: the three kernels run one after another on `stream`;
                                   3: concurrently on internal streams joined back to `stream` */
    int32_t flags;              /* RAWALIGN_FLAG_* */
    int32_t single_max;         /* widest region (levels) swept as one stripe: 2048 or 4096 (0 = 4096).  Regions
                                   of 2049..4096 levels then take one stripe of 34..64 columns per lane (two
                                   waves per SIMD) or two stripes of 17..32 (four waves per SIMD); a query longer
                                   than RAWALIGN_MAX_QUERY_LONG keeps one stripe either way */
    int32_t pipe_waves;         /* RAWALIGN_LONG_PIPELINE: waves per workgroup sharing a pair, 2, 4 or 8 (0 = 4);
                                   long_waves_per_cu then counts waves of that kernel per CU */
} rawalign_opts;

/* Fill `opts` with the library defaults (persistent mode, striped long
 * kernel, occupancy-sized grids, one stream, single stripes up to 4096
 * levels).  Returns RAWALIGN_OK. */
int rawalign_opts_default(rawalign_opts *opts);

/*
 * Plain batched subsequence DTW (Sec. 2.2): one wavefront per pair, pairs
 * taken in arrival order with a static assignment (the baseline).  Three
 * kernels run one after another: regions of at most 2048 levels, of at most
 * 4096 levels, and longer regions.
 *
 *   q, r          device, float32 read events / reference levels
 *   q_size, r_size  number of elements in q and r (bounds for the slices)
 *   q_off, r_off  device, int64 per pair;  q_len, r_len  device, int32 per pair
 *   n_pairs       number of pairs (>= 0; 0 returns at once)
 *   out_score     device, float32 per pair: C_DTW (lower is better)
 *   out_end       device, int32 per pair: 0-based index j into the pair's
 *                 region where the best path ends (smallest on ties)
 *
 * Internal scratch (planning lists, queue counters) is allocated by the
 * library per (device, stream) on first use, grown when a larger batch
 * arrives and kept until process exit.  Calls on one stream are ordered by
 * the stream; calls on different streams use different scratch.  Growing the
 * scratch calls hipMalloc, so a call that may be captured into a HIP graph
 * must follow an uncaptured call of at least the same n_pairs on that stream.
 */
int rawalign_dtw_batch(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                       const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                       int64_t n_pairs, float *out_score, int32_t *out_end, void *stream);

/*
 * Batched subsequence DTW with scheduling options (Sec. 2.2; systems layer):
 * `opts` NULL means the tuned settings for this device if a tuning cache was
 * loaded (rawalign_autotune / rawalign_load_tuning), else the defaults.
 * Persistent mode orders pairs by cell count, longest first, and lets a
 * device-sized grid pull them from an atomic queue.  Arguments as in
 * rawalign_dtw_batch; results are bit-identical to it.
 */
int rawalign_dtw_batch_ex(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                          const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                          int64_t n_pairs, float *out_score, int32_t *out_end, void *stream,
                          const rawalign_opts *opts);

/*
 * Allocation-free batched subsequence DTW, for callers that cannot allocate
 * device memory: code being captured into a HIP graph, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results (bit for bit)
 * and sentinels as rawalign_dtw_batch / rawalign_dtw_batch_ex with default
 * options (persistent queues, striped kernels, every kernel on `stream`),
 * but the planning lists and the multi-stripe kernel's edge slots live in
 * one fixed device array of RAWALIGN_NOALLOC_SCRATCH_BYTES (34 MiB) per
 * GPU, which the library holds from its first use on that GPU until the
 * process ends.  The call makes no hipMalloc, hipFree or other allocating
 * call; the address of the array on the current device is looked up once
 * per device, on the first call there.
 *   - n_pairs > RAWALIGN_NOALLOC_MAX_PAIRS returns RAWALIGN_EINVAL before
 *     anything is enqueued.
 *   - At most RAWALIGN_NOALLOC_EDGE_SLOTS waves sweep regions longer than
 *     4096 levels at once (the other routes use their usual grids), so large
 *     batches of long regions run slower than through rawalign_dtw_batch_ex.
 *   - Every call on one GPU uses the same array, which keeps the last call's
 *     contents (the planning kernels clear what must start at zero).  Calls
 *     that overlap in time on one GPU (on different streams, or from several
 *     threads) race on it and give wrong results: serialise them.
 */
#define RAWALIGN_NOALLOC_MAX_PAIRS 131072
#define RAWALIGN_NOALLOC_EDGE_SLOTS 512
#define RAWALIGN_NOALLOC_SCRATCH_BYTES 35654912
int rawalign_dtw_batch_noalloc(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                               const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                               int64_t n_pairs, float *out_score, int32_t *out_end, void *stream);

/*
 * Streaming extension for Read Until (Sec. 1, Sec. 3.1.2: reads arrive in
 * chunks and a decision is taken after each one).  Job k continues the
 * alignment of one (read, candidate) pair by the events of a new chunk:
 * rows[row_off[k] .. +r_len[k]) holds the last DTW row of the events seen so
 * far (D(N-1, j) for every region level j) and is used as row -1 of the new
 * chunk (its corner D(-1,-1) is +inf); first_chunk[k] != 0 means no events
 * were seen yet and row -1 is all zero (the stored row is not read).  On
 * return the row holds the last row after the chunk, and out_score/out_end
 * are C_DTW and end of the whole prefix seen so far, identical to aligning
 * the concatenated prefix at once.
 *
 *   q, q_size, q_off, q_len  device, the chunk events of every job
 *   r, r_size, r_off, r_len  device, the candidate regions
 *   rows, rows_size          device float32 arena (caller-owned) and its size
 *   row_off                  device int64 per job, start of the job's row
 *   first_chunk              device uint8 per job
 *   n_jobs, out_score, out_end, stream  as above
 * Jobs must not share a row.  A job whose row slice leaves [0, rows_size)
 * gets score NaN, end -2 and its row is untouched.  q_len == 0 leaves the
 * row unchanged and reports the stored row's minimum.
 */
int rawalign_dtw_extend(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                        const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                        float *rows, int64_t rows_size, const int64_t *row_off,
                        const uint8_t *first_chunk, int64_t n_jobs,
                        float *out_score, int32_t *out_end, void *stream, const rawalign_opts *opts);

/*
 * Mapping decision (Sec. 2.3): for read k with candidate pairs
 * cand_off[k] .. cand_off[k]+cand_cnt[k]-1 and n_events[k] aligned events,
 * Score = b_match * N_Read - C_DTW (double precision, from the float C_DTW);
 * the highest score wins (smallest pair index on ties) and the read is mapped
 * iff that score >= threshold.  The paper's defaults are b_match = 0.4 and
 * threshold = 20 (Sec. 3.1.5).  A candidate whose C_DTW is NaN (the sentinel
 * of a pair that was not aligned) is skipped: it cannot win, and it does not
 * hide the candidates after it; a read whose candidates are all NaN gets
 * out_best -1, score -inf, not mapped.
 *   score                     device float32 per pair (C_DTW from a DTW call)
 *   cand_off                  device int64 per read;  cand_cnt, n_events device int32 per read
 *   out_best                  device int32 per read: winning pair index, -1 if no candidates
 *   out_score                 device float64 per read: winning Score, -inf if none
 *   out_mapped                device uint8 per read
 * A read whose candidate range leaves [0, n_pairs) gets out_best -2, score
 * NaN, not mapped.
 */
int rawalign_decide(const float *score, int64_t n_pairs, const int64_t *cand_off, const int32_t *cand_cnt,
                    const int32_t *n_events, int64_t n_reads, double b_match, double threshold,
                    int32_t *out_best, double *out_score, uint8_t *out_mapped, void *stream);

/*
 * Mapping with early termination (Sec. 2.4.1, branch and bound): the same
 * per-read decision as rawalign_dtw_batch followed by rawalign_decide, with
 * hopeless candidates dropped before their table is finished.
 *   - Read k's candidates cand_off[k] .. cand_off[k]+cand_cnt[k]-1 are taken
 *     to be in chaining-score order, best first.  Every read's first
 *     candidate is queued ahead of all other pairs (longest first within
 *     each group); one persistent kernel pulls pairs from that queue, and
 *     waves sweeping a first candidate run at a raised wave priority (their
 *     results bound the other pairs).
 *   - A pair is swept block_rows query rows at a time through its resident
 *     row rows[row_off[p] .. +r_len[p]) (scratch contents).  After a block
 *     that ended at row i the cost of every path is at least min_j D(i, j)
 *     (costs never decrease along a path), so the pair's Score
 *     b_match * n_events[k] - C_DTW is at most b_match * n_events[k] -
 *     min_j D(i, j); when that is strictly below the best Score its read has
 *     reached so far, the pair is dropped: out_score = +inf, out_end = -3.
 *     A completed pair raises its read's best (an atomic maximum).
 *   - A dropped pair can neither win nor tie, so out_best, out_best_score
 *     and out_mapped equal those of rawalign_decide on the scores of the full
 *     computation; completed pairs' out_score/out_end equal
 *     rawalign_dtw_batch's bit for bit.  Which pairs are dropped depends on
 *     timing and can vary between runs.
 *   - max_query: the longest q_len the caller passes; longer pairs get the
 *     sentinel NaN, -2.  block_rows in [64, RAWALIGN_MAX_QUERY_LONG].  A
 *     pair claimed by several reads, or by none, is aligned whole.  rows must
 *     give every pair its own slot of r_len[p] floats.
 *   - opts: long_waves_per_cu sets the persistent grid in waves per CU
 *     (0 = occupancy limit, 16); other fields are not used.  NULL = defaults.
 *   Other arguments, sentinels and limits as in rawalign_dtw_batch and
 *   rawalign_decide.  Scratch (about 9 bytes per pair and 8 per read, plus
 *   the stripe edge slots) is allocated per (device, stream) on first use.
 */
int rawalign_map_bnb(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                     const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len, int64_t n_pairs,
                     const int64_t *cand_off, const int32_t *cand_cnt, const int32_t *n_events, int64_t n_reads,
                     double b_match, double threshold, int32_t max_query, int32_t block_rows,
                     float *rows, int64_t rows_size, const int64_t *row_off,
                     float *out_score, int32_t *out_end, int32_t *out_best, double *out_best_score,
                     uint8_t *out_mapped, void *stream, const rawalign_opts *opts);

/*
 * Subsequence DTW with the start of each alignment.  The paper reports
 * scores by default and can add the alignment path to its output (Sec.
 * 2.4); its first region column is the start.  Two passes over the batch:
 *   1. rawalign_dtw_batch_ex gives out_score (C_DTW) and out_end (e);
 *   2. the reversed query q_{n-1} .. q_0 is aligned against the reversed
 *      region prefix r_e .. r_0, the path anchored at its first cell (the
 *      forward cell (n-1, e)) and free to finish anywhere in the last
 *      reversed row; its best end k (smallest on ties) gives
 *      out_start = e - k.
 * In exact arithmetic this is the largest first column among the optimal
 * paths that end at e (the shortest optimal alignment), and the region
 * interval [start, end] aligned globally costs C_DTW.
 *   Arguments as in rawalign_dtw_batch_ex, plus out_start (device, int32 per
 *   pair).  Pairs without an end keep its sentinel as their start (-1
 *   degenerate, -2 invalid).  opts: as in rawalign_dtw_batch_ex (NULL = tuned
 *   or defaults) for both passes; long_kernel must be RAWALIGN_LONG_STRIPED.
 *   Scratch: that of rawalign_dtw_batch plus 12 bytes per pair, per (device,
 *   stream).  The reverse pass sweeps sum(e + 1) * n cells.
 */
int rawalign_dtw_span(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                      const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                      int64_t n_pairs, float *out_score, int32_t *out_end, int32_t *out_start, void *stream,
                      const rawalign_opts *opts);

/*
 * Subsequence DTW with the warping path of every alignment (Sec. 2.4: the
 * alignment path as an optional output).  First as rawalign_dtw_span (score,
 * end e, start s); then the path is an optimal global path from (0, s) to
 * (n-1, e), i.e. global DTW of the whole query against r[s..e] entered from
 * the corner D(-1, s-1) = 0, with ties between the neighbours resolved
 * north-west first, then north, then west when the path is read back from
 * (n-1, e).  A monotone path covers a contiguous range of every row:
 *   path_off   device int64 per pair: offset of the pair's n entries in
 *              path_lo / path_hi (caller-owned, path_size entries each)
 *   path_lo[path_off[p] + i], path_hi[path_off[p] + i]
 *              the first and last region columns that read event i is
 *              aligned with (region indices, like end and start):
 *              path_lo[off] = start, path_hi[off + n - 1] = end.
 *   dirs, dir_off, dir_size
 *              caller-owned device workspace of dir_size 64-bit words; pair
 *              p uses the words from dir_off[p] on, n * (64 * S + 1) of them
 *              for an interval of L = e - s + 1 levels, S = ceil(L / 2048)
 *              (2 bits per cell and a stripe edge).  The interval is at most
 *              m levels, so n * (64 * ceil(m / 2048) + 1) words always
 *              suffice; a caller that first calls rawalign_dtw_span can size
 *              every range from its interval exactly and pass
 *              RAWALIGN_FLAG_SPAN_GIVEN with that call's outputs.  A pair
 *              whose range does not hold its interval gets -4 in every
 *              entry.  The ranges of the pairs of one call must not overlap.
 *   Pairs without an alignment get their end sentinel in every entry (-1
 *   empty region, -2 invalid slice); an empty query has no entries.
 *   Entries of a pair whose range leaves [0, path_size) are not written.
 *   opts->flags & RAWALIGN_FLAG_SPAN_GIVEN: out_score, out_end and
 *   out_start are inputs, the result of rawalign_dtw_span on the same pairs
 *   (an end or start that no alignment of the pair can have gets -2 in
 *   every entry); the span passes are skipped.
 *   Other arguments, opts and errors as in rawalign_dtw_span; beyond that
 *   call's scratch this entry point allocates nothing.  One wave per pair
 *   records the directions stripe by stripe in the lane-striped order of the
 *   other kernels; one thread per pair then follows them back.
 */
int rawalign_dtw_path(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                      const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                      int64_t n_pairs, const int64_t *dir_off, uint64_t *dirs, int64_t dir_size,
                      const int64_t *path_off, int32_t *path_lo, int32_t *path_hi, int64_t path_size,
                      float *out_score, int32_t *out_end, int32_t *out_start, void *stream,
                      const rawalign_opts *opts);

/*
 * Banded subsequence DTW (Sec. 2.4.3): only the cells near the diagonal of
 * slope n/m are computed.  Row i's diagonal column is c(i) = floor(i*m/n);
 * cell (i, j) is in the band iff |j - c(i)| <= band[p] (half-width in
 * levels; 20% of the fragment, the paper's default, is about 0.2*m); other
 * cells are +inf.  Row -1 is the free start, and the result is the minimum
 * over the band cells of row n-1 (smallest j), +inf with end -1 when none is
 * reachable.  band[p] >= m-1 gives plain subsequence DTW.
 *   Arguments as in rawalign_dtw_batch, plus band (device, int32 per pair).
 *   One wave per pair in a band-relative frame (frame positions follow the
 *   diagonal) when m <= n (at least as many events as levels, as in a
 *   chained segment: about 3.3 events per level) and 2*min(band, m-1)+1 <=
 *   2048.  Other pairs use frames over the whole region with the cells
 *   outside the band forced to +inf: one stripe up to 2048 levels, else
 *   stripes of up to 2048 columns swept one after another, each over only
 *   the rows the band spends in it.  The pairs are planned on the device
 *   into four classes (band frames up to 512 columns, wider band frames,
 *   one whole-region stripe, several stripes), each taken longest first
 *   from a persistent queue; the class kernels run concurrently on internal
 *   streams joined back to `stream`.  Scratch: that of rawalign_dtw_batch
 *   plus stripe edge slots, per (device, stream).
 *   A query longer than RAWALIGN_MAX_QUERY_LONG against more than 2048
 *   levels with a band wider than 2048 columns (the one shape no class
 *   takes) gets the sentinel NaN, end -4.  A negative band or an invalid
 *   slice gives NaN, -2; n == 0 gives (0, -1), m == 0 (+inf, -1).
 */
int rawalign_dtw_band(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                      const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                      const int32_t *band, int64_t n_pairs, float *out_score, int32_t *out_end, void *stream);

/*
 * Global DTW between two anchors (Sec. 2.4.2, anchor-guided alignment): a
 * chain's anchors sit at the upper-left and lower-right corners of every gap
 * between them, and the signals they cover are not aligned again, so the
 * path enters the gap at (0, 0) from the corner D(-1,-1) = 0 and leaves at
 * (n-1, m-1); the rest of row -1 and of column -1 is +inf.
 *   Arguments as in rawalign_dtw_batch (device pointers, per-pair offset and
 *   length), with
 *   out_score  device float32 per pair: D(n-1, m-1)
 *   out_end    device int32 per pair, may be NULL: m-1 (-1 for the
 *              degenerate pairs below)
 *   opts       mode, streams and grids as in rawalign_dtw_batch_ex;
 *              long_kernel must be RAWALIGN_LONG_STRIPED; NULL = defaults
 *              for anchor gaps: three streams, one persistent wave per CU
 *              for regions above 2048 levels (not the tuned settings)
 * Pairs of at most 64 levels are aligned one pair per lane (grouped on the
 * device into 8 width classes, longest queries first); wider ones by the
 * striped kernels.  With three streams the call forks before planning: the
 * width-class planning and the width classes run on internal streams, the
 * striped routes on `stream` itself, all concurrently, joined back to
 * `stream` before the call returns its work to it.
 * Degenerate pairs: n == m == 0 (the anchors touch diagonally) costs 0;
 * n == 0 or m == 0 alone costs +inf (no path through the gap's own cells).
 * Invalid slices get NaN (end -2), as in rawalign_dtw_batch.  Scratch as in
 * rawalign_dtw_batch, plus 32 bytes per pair for the per-lane planning (one
 * record per gap).
 */
int rawalign_dtw_global_batch(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                              const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                              int64_t n_pairs, float *out_score, int32_t *out_end, void *stream,
                              const rawalign_opts *opts);

/*
 * Chain sums and the mapping decision over anchored candidates (Sec. 2.4.2
 * with Sec. 2.3):
 *   - chain c owns gaps chain_gap_off[c] .. +chain_gap_cnt[c]; its cost is
 *     the float sum of those gaps' costs, added in gap order
 *     (out_chain_cost; 0 without gaps, NaN if the range leaves [0, n_gaps));
 *   - read k owns chains cand_off[k] .. +cand_cnt[k]; chain c scores
 *     b_match * chain_events[c] - cost (double), where chain_events counts
 *     the read events the chain aligns; the highest score wins (smallest
 *     chain index on ties) and the read is mapped iff it is >= threshold;
 *     a chain whose cost is NaN is skipped, as in rawalign_decide.
 *   gap_cost (n_gaps floats, e.g. from rawalign_dtw_global_batch),
 *   chain_gap_off int64, chain_gap_cnt/chain_events int32 per chain,
 *   cand_off int64, cand_cnt int32 per read; outputs as in rawalign_decide
 *   (out_best is a chain index).  All device pointers, async on `stream`.
 */
int rawalign_chain_decide(const float *gap_cost, int64_t n_gaps, const int64_t *chain_gap_off,
                          const int32_t *chain_gap_cnt, const int32_t *chain_events, int64_t n_chains,
                          const int64_t *cand_off, const int32_t *cand_cnt, int64_t n_reads, double b_match,
                          double threshold, float *out_chain_cost, int32_t *out_best, double *out_best_score,
                          uint8_t *out_mapped, void *stream);

/*
 * Autotuner: times candidate settings of rawalign_dtw_batch_ex on the
 * caller's device batch (same layout as rawalign_dtw_batch; out_score and
 * out_end are scratch outputs) and keeps the fastest as this device's tuned
 * setting, which opts == NULL then selects.  Two stages, each candidate one
 * warm-up call and the mean of three:
 *   1. the kernel shape: the single-stripe cut-off (single_max 4096 or 2048,
 *      i.e. 34..64 columns per lane on one stripe or 17..32 on two for
 *      regions of 2049..4096 levels) times the long-route kernel and its
 *      workgroup shape (one wave per pair, 2, 4 or 8 waves sharing each
 *      pair: RAWALIGN_LONG_PIPELINE, or one 256-thread workgroup per pair:
 *      RAWALIGN_LONG_ANTIDIAG);
 *   2. at that shape: one or three streams, and each route's persistent grid
 *      at or below its occupancy limit.
 * Every candidate returns the same bits, so the choice affects time only.
 * The anti-diagonal kernel serves plain batches only: calls of the other
 * entry points that inherit a tuned setting naming it (opts NULL) take the
 * striped kernel at its default grid instead; explicit opts naming it are
 * rejected there as before.
 * If cache_path is not NULL the result is also written there as JSON keyed
 * by device name, gfx architecture and library version (rawalign_load_tuning
 * reads it back).  `best` (host, may be NULL) receives it.  The batch should
 * have the size distribution of the work to come (the tuner measures, it
 * does not model).  Synchronises `stream`.
 */
int rawalign_autotune(const float *q, int64_t q_size, const int64_t *q_off, const int32_t *q_len,
                      const float *r, int64_t r_size, const int64_t *r_off, const int32_t *r_len,
                      int64_t n_pairs, float *out_score, int32_t *out_end, void *stream,
                      const char *cache_path, rawalign_opts *best);

/* Load a tuning cache written by rawalign_autotune; entries for other
 * devices or library versions are ignored (returns RAWALIGN_EINVAL then). */
int rawalign_load_tuning(const char *cache_path, rawalign_opts *out);

/* Per-kernel timing of the last call made with RAWALIGN_FLAG_TIMING. */
typedef struct rawalign_timing {
    float plan_ms;    /* routing / ordering kernels */
    float lo_ms;      /* regions <= 2048 levels */
    float hi_ms;      /* regions 2049..4096 levels */
    float long_ms;    /* regions > 4096 levels */
    float total_ms;   /* first to last event of the call */
} rawalign_timing;
int rawalign_last_timing(rawalign_timing *out);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *rawalign_last_error(void);

/* Library version string. */
const char *rawalign_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RAWALIGN_H */
