/*
 * dtw_oracle.c -- CPU oracle for subsequence dynamic time warping (DTW).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (the HIP library) shares no code, header, table or helper with it.
 *
 * What it computes (RawAlign, arXiv 2310.05037, Sec. 2.2 "Alignment via
 * Dynamic Time Warping"): a two-dimensional dynamic-programming table in
 * which every entry adds the numerical difference of the two signal values
 * (no fixed indel penalty) to the smallest of its north, north-west and west
 * neighbours.  The paper aligns a read's events against a candidate region
 * that is longer than the read, so the query must be aligned whole while the
 * alignment may start and end anywhere in the region (subsequence DTW, the
 * textbook form in Mueller, "Fundamentals of Music Processing", 2015, Ch. 7):
 *
 *   c(i,j)  = |q_i - r_j|                 (float inputs widened exactly)
 *   D(-1,j) = 0          for j = -1..m-1  (free start anywhere in the region)
 *   D(i,-1) = +inf       for i >= 0
 *   D(i,j)  = c(i,j) + min{ D(i-1,j-1), D(i-1,j), D(i,j-1) }
 *   C_DTW   = min_j D(n-1,j),   end = smallest j attaining it.
 *
 * Degenerate inputs: n == 0 gives cost 0 and end -1; m == 0 (with n > 0)
 * gives cost +inf and end -1.
 *
 * Streaming (Read Until chunks, Sec. 1 and Sec. 3.1.2): when a previous
 * chunk's last row is supplied as row -1, D(-1,j) = row[j] for j >= 0 and the
 * corner D(-1,-1) is +inf, because column -1 is +inf for every real row.
 * The result then equals the definition applied to the concatenated prefix.
 *
 * Precision: the reference is double precision.  A float instantiation of
 * the same recurrence is provided as well: every cell is one rounded
 * subtraction, an exact absolute value, an exact minimum and one rounded
 * addition, so any evaluation order of the table gives bit-identical float
 * results, which makes the float version a bitwise check for GPU code.
 * Build without -ffast-math and without floating-point contraction.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double min3_d(double a, double b, double c)
{
    double x = a < b ? a : b;
    return x < c ? x : c;
}

static float min3_f(float a, float b, float c)
{
    float x = a < b ? a : b;
    return x < c ? x : c;
}

/*
 * One pair in double precision.
 *   q[0..n), r[0..m): inputs (float, widened to double).
 *   init_row: NULL for a fresh alignment (row -1 all zero), else the m
 *             values of the previous chunk's last row (corner +inf).
 *   last_row: optional output, the m values of row n-1 (or of row -1 when
 *             n == 0).
 *   end:      output, smallest j of the minimum in row n-1 (-1 if none).
 * Returns C_DTW.  Returns NaN and end = -2 if memory runs out.
 */
double oracle_dtw_f64(const float *q, int64_t n, const float *r, int64_t m,
                      const double *init_row, double *last_row, int32_t *end)
{
    if (m == 0) {
        *end = -1;
        return n == 0 ? 0.0 : INFINITY;
    }
    /* prev[j+1] holds D(i-1, j); prev[0] holds D(i-1, -1). */
    double *prev = malloc((size_t)(m + 1) * sizeof(double));
    double *cur = malloc((size_t)(m + 1) * sizeof(double));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        *end = -2;
        return NAN;
    }
    if (init_row) {
        prev[0] = INFINITY;
        for (int64_t j = 0; j < m; ++j)
            prev[j + 1] = init_row[j];
    } else {
        for (int64_t j = 0; j <= m; ++j)
            prev[j] = 0.0;
    }
    for (int64_t i = 0; i < n; ++i) {
        cur[0] = INFINITY; /* D(i, -1) */
        double qi = (double)q[i];
        for (int64_t j = 0; j < m; ++j) {
            double c = fabs(qi - (double)r[j]);
            cur[j + 1] = c + min3_d(prev[j], prev[j + 1], cur[j]);
        }
        double *t = prev;
        prev = cur;
        cur = t;
    }
    double best;
    int32_t arg;
    if (n == 0 && !init_row) {
        best = 0.0;
        arg = -1;
    } else {
        best = prev[1];
        arg = 0;
        for (int64_t j = 1; j < m; ++j) {
            if (prev[j + 1] < best) {
                best = prev[j + 1];
                arg = (int32_t)j;
            }
        }
    }
    if (last_row)
        for (int64_t j = 0; j < m; ++j)
            last_row[j] = prev[j + 1];
    free(prev);
    free(cur);
    *end = arg;
    return best;
}

/* The same recurrence with every value held in float. */
float oracle_dtw_f32(const float *q, int64_t n, const float *r, int64_t m,
                     const float *init_row, float *last_row, int32_t *end)
{
    if (m == 0) {
        *end = -1;
        return n == 0 ? 0.0f : INFINITY;
    }
    float *prev = malloc((size_t)(m + 1) * sizeof(float));
    float *cur = malloc((size_t)(m + 1) * sizeof(float));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        *end = -2;
        return NAN;
    }
    if (init_row) {
        prev[0] = INFINITY;
        for (int64_t j = 0; j < m; ++j)
            prev[j + 1] = init_row[j];
    } else {
        for (int64_t j = 0; j <= m; ++j)
            prev[j] = 0.0f;
    }
    for (int64_t i = 0; i < n; ++i) {
        cur[0] = INFINITY;
        float qi = q[i];
        for (int64_t j = 0; j < m; ++j) {
            float d = qi - r[j];
            float c = fabsf(d);
            cur[j + 1] = c + min3_f(prev[j], prev[j + 1], cur[j]);
        }
        float *t = prev;
        prev = cur;
        cur = t;
    }
    float best;
    int32_t arg;
    if (n == 0 && !init_row) {
        best = 0.0f;
        arg = -1;
    } else {
        best = prev[1];
        arg = 0;
        for (int64_t j = 1; j < m; ++j) {
            if (prev[j + 1] < best) {
                best = prev[j + 1];
                arg = (int32_t)j;
            }
        }
    }
    if (last_row)
        for (int64_t j = 0; j < m; ++j)
            last_row[j] = prev[j + 1];
    free(prev);
    free(cur);
    *end = arg;
    return best;
}

/*
 * Full table D(i,j), row-major n x m, double precision, fresh alignment.
 * For small inputs in tests of the table's own invariants.
 */
void oracle_dtw_matrix_f64(const float *q, int64_t n, const float *r, int64_t m,
                           double *D)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            double diag = (i == 0) ? 0.0 : (j == 0 ? INFINITY : D[(i - 1) * m + j - 1]);
            double up = (i == 0) ? 0.0 : D[(i - 1) * m + j];
            double left = (j == 0) ? INFINITY : D[i * m + j - 1];
            double c = fabs((double)q[i] - (double)r[j]);
            D[i * m + j] = c + min3_d(diag, up, left);
        }
    }
}

/*
 * Global DTW between two anchors (Sec. 2.4.2, anchor-guided alignment).  The
 * anchors of a chain are the cells at the upper-left and lower-right corners
 * of a gap's table; the signals they cover are not aligned again.  So the
 * path enters the gap diagonally from the upper-left anchor and leaves it
 * diagonally into the lower-right one:
 *
 *   D(-1,-1) = 0,  D(-1,j) = +inf (j >= 0),  D(i,-1) = +inf (i >= 0)
 *   D(i,j)   = c(i,j) + min{ D(i-1,j-1), D(i-1,j), D(i,j-1) }
 *   G        = D(n-1, m-1)
 *
 * Degenerate gaps: n == m == 0 (the anchors touch diagonally) costs 0; a gap
 * with events but no levels, or levels but no events, has no path through
 * its own cells and costs +inf.  Returns NaN if memory runs out.
 */
double oracle_dtw_global_f64(const float *q, int64_t n, const float *r, int64_t m)
{
    if (n == 0 || m == 0)
        return (n == 0 && m == 0) ? 0.0 : INFINITY;
    double *prev = malloc((size_t)(m + 1) * sizeof(double));
    double *cur = malloc((size_t)(m + 1) * sizeof(double));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return NAN;
    }
    /* prev[j+1] = D(i-1, j); prev[0] = D(i-1, -1). */
    prev[0] = 0.0; /* the corner D(-1,-1) */
    for (int64_t j = 0; j < m; ++j)
        prev[j + 1] = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        cur[0] = INFINITY;
        double qi = (double)q[i];
        for (int64_t j = 0; j < m; ++j) {
            double c = fabs(qi - (double)r[j]);
            cur[j + 1] = c + min3_d(prev[j], prev[j + 1], cur[j]);
        }
        double *t = prev;
        prev = cur;
        cur = t;
    }
    double g = prev[m];
    free(prev);
    free(cur);
    return g;
}

/* The same recurrence with every value held in float. */
float oracle_dtw_global_f32(const float *q, int64_t n, const float *r, int64_t m)
{
    if (n == 0 || m == 0)
        return (n == 0 && m == 0) ? 0.0f : INFINITY;
    float *prev = malloc((size_t)(m + 1) * sizeof(float));
    float *cur = malloc((size_t)(m + 1) * sizeof(float));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return NAN;
    }
    prev[0] = 0.0f;
    for (int64_t j = 0; j < m; ++j)
        prev[j + 1] = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        cur[0] = INFINITY;
        float qi = q[i];
        for (int64_t j = 0; j < m; ++j) {
            float d = qi - r[j];
            float c = fabsf(d);
            cur[j + 1] = c + min3_f(prev[j], prev[j + 1], cur[j]);
        }
        float *t = prev;
        prev = cur;
        cur = t;
    }
    float g = prev[m];
    free(prev);
    free(cur);
    return g;
}

/*
 * Start of the alignment.  The paper's DTW reports a score by default and
 * can add the alignment path to its output (Sec. 2.4); the path's first
 * region column is its start.  Given the end column e of the subsequence
 * recurrence above, the read is aligned backwards: the reversed query
 * q_{n-1} .. q_0 against the reversed region prefix r_e .. r_0, the path
 * anchored at its first cell (the forward cell (n-1, e)) and free to finish
 * anywhere in the last reversed row (forward row 0):
 *
 *   R(-1,-1) = 0,  R(-1,k) = +inf (k >= 0),  R(i,-1) = +inf (i >= 0)
 *   R(i,k)   = |q_{n-1-i} - r_{e-k}| + min{ R(i-1,k-1), R(i-1,k), R(i,k-1) }
 *   k*       = smallest k minimising R(n-1, k),   start = e - k*
 *
 * A reversed path is a forward path read backwards, so min_k R(n-1, k) is
 * C_DTW in exact arithmetic, and k* picks the largest first column among
 * the optimal paths that end at e: the shortest optimal alignment.  The
 * same steps in float give the float start.
 *
 * Degenerate pairs: end -1 (empty query or region) gives start -1.
 */
static int32_t rev_argmin_f64(const float *q, int64_t n, const float *r, int32_t e)
{
    int64_t m = (int64_t)e + 1;
    double *prev = malloc((size_t)(m + 1) * sizeof(double));
    double *cur = malloc((size_t)(m + 1) * sizeof(double));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return -2;
    }
    prev[0] = 0.0; /* R(-1,-1): the anchored first cell */
    for (int64_t k = 0; k < m; ++k)
        prev[k + 1] = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        cur[0] = INFINITY;
        double qi = (double)q[n - 1 - i];
        for (int64_t k = 0; k < m; ++k) {
            double c = fabs(qi - (double)r[e - k]);
            cur[k + 1] = c + min3_d(prev[k], prev[k + 1], cur[k]);
        }
        double *t = prev;
        prev = cur;
        cur = t;
    }
    int32_t arg = 0;
    double best = prev[1];
    for (int64_t k = 1; k < m; ++k) {
        if (prev[k + 1] < best) {
            best = prev[k + 1];
            arg = (int32_t)k;
        }
    }
    free(prev);
    free(cur);
    return arg;
}

static int32_t rev_argmin_f32(const float *q, int64_t n, const float *r, int32_t e)
{
    int64_t m = (int64_t)e + 1;
    float *prev = malloc((size_t)(m + 1) * sizeof(float));
    float *cur = malloc((size_t)(m + 1) * sizeof(float));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return -2;
    }
    prev[0] = 0.0f;
    for (int64_t k = 0; k < m; ++k)
        prev[k + 1] = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        cur[0] = INFINITY;
        float qi = q[n - 1 - i];
        for (int64_t k = 0; k < m; ++k) {
            float d = qi - r[e - k];
            float c = fabsf(d);
            cur[k + 1] = c + min3_f(prev[k], prev[k + 1], cur[k]);
        }
        float *t = prev;
        prev = cur;
        cur = t;
    }
    int32_t arg = 0;
    float best = prev[1];
    for (int64_t k = 1; k < m; ++k) {
        if (prev[k + 1] < best) {
            best = prev[k + 1];
            arg = (int32_t)k;
        }
    }
    free(prev);
    free(cur);
    return arg;
}

/*
 * The warping path of an alignment (Sec. 2.4: the path can be added to the
 * output).  Given the alignment's start s and end e (oracle_dtw_span_*), the
 * path is an optimal global path from (0, s) to (n-1, e): global DTW of the
 * whole query against r[s..e], entered from the corner D(-1, s-1) = 0 and
 * left at (n-1, e).  Every cell records which neighbour gave its minimum,
 * preferring the north-west one, then the north, then the west on ties, and
 * the path is read back from (n-1, e).  A monotone path covers a contiguous
 * column range in every row: lo[i] .. hi[i] (region indices) are the levels
 * that read event i is aligned with.  Returns the path's cost (the global
 * cost of [s, e]); NAN if memory runs out.
 */
#define PATH_NW 0
#define PATH_N 1
#define PATH_W 2

static void path_trace(const unsigned char *dir, int64_t n, int64_t L, int32_t s, int32_t *lo, int32_t *hi)
{
    int64_t i = n - 1, j = L - 1;
    hi[i] = (int32_t)(s + j);
    for (;;) {
        lo[i] = (int32_t)(s + j);
        if (i == 0 && j == 0)
            break;
        unsigned char d = dir[i * L + j];
        if (d == PATH_W) {
            --j;
        } else {
            if (d == PATH_NW)
                --j;
            --i;
            hi[i] = (int32_t)(s + j);
        }
    }
}

double oracle_dtw_path_f64(const float *q, int64_t n, const float *r, int32_t s, int32_t e, int32_t *lo,
                           int32_t *hi)
{
    int64_t L = (int64_t)e - s + 1;
    double *prev = malloc((size_t)(L + 1) * sizeof(double));
    double *cur = malloc((size_t)(L + 1) * sizeof(double));
    unsigned char *dir = malloc((size_t)(n * L));
    if (!prev || !cur || !dir) {
        free(prev);
        free(cur);
        free(dir);
        return NAN;
    }
    prev[0] = 0.0; /* the corner D(-1, s-1) */
    for (int64_t j = 0; j < L; ++j)
        prev[j + 1] = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        cur[0] = INFINITY;
        double qi = (double)q[i];
        for (int64_t j = 0; j < L; ++j) {
            double nw = prev[j], no = prev[j + 1], we = cur[j];
            double mn = min3_d(nw, no, we);
            dir[i * L + j] = nw == mn ? PATH_NW : (no == mn ? PATH_N : PATH_W);
            cur[j + 1] = fabs(qi - (double)r[s + j]) + mn;
        }
        double *t = prev;
        prev = cur;
        cur = t;
    }
    double g = prev[L];
    path_trace(dir, n, L, s, lo, hi);
    free(prev);
    free(cur);
    free(dir);
    return g;
}

float oracle_dtw_path_f32(const float *q, int64_t n, const float *r, int32_t s, int32_t e, int32_t *lo,
                          int32_t *hi)
{
    int64_t L = (int64_t)e - s + 1;
    float *prev = malloc((size_t)(L + 1) * sizeof(float));
    float *cur = malloc((size_t)(L + 1) * sizeof(float));
    unsigned char *dir = malloc((size_t)(n * L));
    if (!prev || !cur || !dir) {
        free(prev);
        free(cur);
        free(dir);
        return NAN;
    }
    prev[0] = 0.0f;
    for (int64_t j = 0; j < L; ++j)
        prev[j + 1] = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        cur[0] = INFINITY;
        float qi = q[i];
        for (int64_t j = 0; j < L; ++j) {
            float nw = prev[j], no = prev[j + 1], we = cur[j];
            float mn = min3_f(nw, no, we);
            dir[i * L + j] = nw == mn ? PATH_NW : (no == mn ? PATH_N : PATH_W);
            float d = qi - r[s + j];
            cur[j + 1] = fabsf(d) + mn;
        }
        float *t = prev;
        prev = cur;
        cur = t;
    }
    float g = prev[L];
    path_trace(dir, n, L, s, lo, hi);
    free(prev);
    free(cur);
    free(dir);
    return g;
}

/* Subsequence DTW with its start: returns C_DTW, writes end and start. */
double oracle_dtw_span_f64(const float *q, int64_t n, const float *r, int64_t m, int32_t *end, int32_t *start)
{
    double c = oracle_dtw_f64(q, n, r, m, NULL, NULL, end);
    if (*end < 0) {
        *start = *end;
        return c;
    }
    int32_t k = rev_argmin_f64(q, n, r, *end);
    *start = k < 0 ? k : *end - k;
    return c;
}

float oracle_dtw_span_f32(const float *q, int64_t n, const float *r, int64_t m, int32_t *end, int32_t *start)
{
    float c = oracle_dtw_f32(q, n, r, m, NULL, NULL, end);
    if (*end < 0) {
        *start = *end;
        return c;
    }
    int32_t k = rev_argmin_f32(q, n, r, *end);
    *start = k < 0 ? k : *end - k;
    return c;
}

/*
 * Banded subsequence DTW (Sec. 2.4.3): only cells near the diagonal of slope
 * n/m are computed, the band following that diagonal rather than the slope 1
 * one.  Reading: the diagonal column of row i is c(i) = floor(i*m/n); a
 * cell (i,j) is in the band iff |j - c(i)| <= w (half-width w >= 0, in
 * levels; a band w = 0.2*m wide on each side is 0.2*n rows from the
 * diagonal, the paper's 20% of the fragment).  Cells outside the band are
 * +inf; row -1 stays the free start (all zero) and column -1 +inf; the
 * result is the minimum over row n-1 (band cells only), smallest j; +inf and
 * end -1 when no cell of row n-1 is reachable.  n == 0: (0, -1); m == 0:
 * (+inf, -1).  w >= m-1 puts every cell in the band: plain subsequence DTW.
 */
double oracle_dtw_band_f64(const float *q, int64_t n, const float *r, int64_t m, int64_t w, int32_t *end)
{
    if (n == 0 || m == 0) {
        *end = -1;
        return n == 0 ? 0.0 : INFINITY;
    }
    double *prev = malloc((size_t)(m + 1) * sizeof(double));
    double *cur = malloc((size_t)(m + 1) * sizeof(double));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        *end = -2;
        return NAN;
    }
    for (int64_t j = 0; j <= m; ++j)
        prev[j] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = i * m / n;
        cur[0] = INFINITY;
        double qi = (double)q[i];
        for (int64_t j = 0; j < m; ++j) {
            if (j < c - w || j > c + w) {
                cur[j + 1] = INFINITY;
                continue;
            }
            double d = fabs(qi - (double)r[j]);
            cur[j + 1] = d + min3_d(prev[j], prev[j + 1], cur[j]);
        }
        double *t = prev;
        prev = cur;
        cur = t;
    }
    double best = INFINITY;
    int32_t arg = -1;
    for (int64_t j = 0; j < m; ++j) {
        if (prev[j + 1] < best) {
            best = prev[j + 1];
            arg = (int32_t)j;
        }
    }
    free(prev);
    free(cur);
    *end = arg;
    return best;
}

float oracle_dtw_band_f32(const float *q, int64_t n, const float *r, int64_t m, int64_t w, int32_t *end)
{
    if (n == 0 || m == 0) {
        *end = -1;
        return n == 0 ? 0.0f : INFINITY;
    }
    float *prev = malloc((size_t)(m + 1) * sizeof(float));
    float *cur = malloc((size_t)(m + 1) * sizeof(float));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        *end = -2;
        return NAN;
    }
    for (int64_t j = 0; j <= m; ++j)
        prev[j] = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = i * m / n;
        cur[0] = INFINITY;
        float qi = q[i];
        for (int64_t j = 0; j < m; ++j) {
            if (j < c - w || j > c + w) {
                cur[j + 1] = INFINITY;
                continue;
            }
            float d = qi - r[j];
            float a = fabsf(d);
            cur[j + 1] = a + min3_f(prev[j], prev[j + 1], cur[j]);
        }
        float *t = prev;
        prev = cur;
        cur = t;
    }
    float best = INFINITY;
    int32_t arg = -1;
    for (int64_t j = 0; j < m; ++j) {
        if (prev[j + 1] < best) {
            best = prev[j + 1];
            arg = (int32_t)j;
        }
    }
    free(prev);
    free(cur);
    *end = arg;
    return best;
}

/* ---- batches: pairs are independent, threads take pairs from a counter ---- */

struct batch_job {
    const float *q;
    const int64_t *q_off;
    const int32_t *q_len;
    const float *r;
    const int64_t *r_off;
    const int32_t *r_len;
    int64_t n_pairs;
    double *out64;
    float *out32;
    int32_t *out_end;   /* NULL for global alignment (no end column) */
    int global;
    int32_t *out_start; /* span: start column per pair */
    const int32_t *band; /* banded: half-width per pair */
    int64_t next;
};

static void *batch_worker(void *arg)
{
    struct batch_job *job = arg;
    for (;;) {
        int64_t p = __atomic_fetch_add(&job->next, 1, __ATOMIC_RELAXED);
        if (p >= job->n_pairs)
            break;
        const float *qp = job->q + job->q_off[p];
        const float *rp = job->r + job->r_off[p];
        if (job->band) {
            if (job->out64)
                job->out64[p] = oracle_dtw_band_f64(qp, job->q_len[p], rp, job->r_len[p], job->band[p],
                                                    &job->out_end[p]);
            else
                job->out32[p] = oracle_dtw_band_f32(qp, job->q_len[p], rp, job->r_len[p], job->band[p],
                                                    &job->out_end[p]);
        } else if (job->out_start) {
            if (job->out64)
                job->out64[p] = oracle_dtw_span_f64(qp, job->q_len[p], rp, job->r_len[p], &job->out_end[p],
                                                    &job->out_start[p]);
            else
                job->out32[p] = oracle_dtw_span_f32(qp, job->q_len[p], rp, job->r_len[p], &job->out_end[p],
                                                    &job->out_start[p]);
        } else if (job->global) {
            if (job->out64)
                job->out64[p] = oracle_dtw_global_f64(qp, job->q_len[p], rp, job->r_len[p]);
            else
                job->out32[p] = oracle_dtw_global_f32(qp, job->q_len[p], rp, job->r_len[p]);
        } else if (job->out64)
            job->out64[p] = oracle_dtw_f64(qp, job->q_len[p], rp, job->r_len[p],
                                           NULL, NULL, &job->out_end[p]);
        else
            job->out32[p] = oracle_dtw_f32(qp, job->q_len[p], rp, job->r_len[p],
                                           NULL, NULL, &job->out_end[p]);
    }
    return NULL;
}

static int run_batch(struct batch_job *job, int n_threads)
{
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > 256)
        n_threads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 1; t < n_threads; ++t) {
        if (pthread_create(&th[started], NULL, batch_worker, job) != 0)
            break;
        ++started;
    }
    batch_worker(job);
    for (int t = 0; t < started; ++t)
        pthread_join(th[t], NULL);
    return started + 1; /* threads that actually worked */
}

/*
 * Pair p aligns q[q_off[p] .. +q_len[p]) against r[r_off[p] .. +r_len[p]).
 * Returns the number of threads used.
 */
int oracle_dtw_batch_f64(const float *q, const int64_t *q_off, const int32_t *q_len,
                         const float *r, const int64_t *r_off, const int32_t *r_len,
                         int64_t n_pairs, double *out_score, int32_t *out_end,
                         int n_threads)
{
    struct batch_job job = {q, q_off, q_len, r, r_off, r_len, n_pairs,
                            out_score, NULL, out_end, 0, NULL, NULL, 0};
    return run_batch(&job, n_threads);
}

int oracle_dtw_batch_f32(const float *q, const int64_t *q_off, const int32_t *q_len,
                         const float *r, const int64_t *r_off, const int32_t *r_len,
                         int64_t n_pairs, float *out_score, int32_t *out_end,
                         int n_threads)
{
    struct batch_job job = {q, q_off, q_len, r, r_off, r_len, n_pairs,
                            NULL, out_score, out_end, 0, NULL, NULL, 0};
    return run_batch(&job, n_threads);
}

/* Global DTW (corner entry and exit) of every pair; no end column. */
int oracle_dtw_global_batch_f64(const float *q, const int64_t *q_off, const int32_t *q_len,
                                const float *r, const int64_t *r_off, const int32_t *r_len,
                                int64_t n_pairs, double *out_score, int n_threads)
{
    struct batch_job job = {q, q_off, q_len, r, r_off, r_len, n_pairs,
                            out_score, NULL, NULL, 1, NULL, NULL, 0};
    return run_batch(&job, n_threads);
}

int oracle_dtw_global_batch_f32(const float *q, const int64_t *q_off, const int32_t *q_len,
                                const float *r, const int64_t *r_off, const int32_t *r_len,
                                int64_t n_pairs, float *out_score, int n_threads)
{
    struct batch_job job = {q, q_off, q_len, r, r_off, r_len, n_pairs,
                            NULL, out_score, NULL, 1, NULL, NULL, 0};
    return run_batch(&job, n_threads);
}

/* Subsequence DTW with start and end of every pair. */
int oracle_dtw_span_batch_f64(const float *q, const int64_t *q_off, const int32_t *q_len,
                              const float *r, const int64_t *r_off, const int32_t *r_len,
                              int64_t n_pairs, double *out_score, int32_t *out_end, int32_t *out_start,
                              int n_threads)
{
    struct batch_job job = {q, q_off, q_len, r, r_off, r_len, n_pairs,
                            out_score, NULL, out_end, 0, out_start, NULL, 0};
    return run_batch(&job, n_threads);
}

int oracle_dtw_span_batch_f32(const float *q, const int64_t *q_off, const int32_t *q_len,
                              const float *r, const int64_t *r_off, const int32_t *r_len,
                              int64_t n_pairs, float *out_score, int32_t *out_end, int32_t *out_start,
                              int n_threads)
{
    struct batch_job job = {q, q_off, q_len, r, r_off, r_len, n_pairs,
                            NULL, out_score, out_end, 0, out_start, NULL, 0};
    return run_batch(&job, n_threads);
}

/* Banded subsequence DTW of every pair (band: half-width per pair). */
int oracle_dtw_band_batch_f64(const float *q, const int64_t *q_off, const int32_t *q_len,
                              const float *r, const int64_t *r_off, const int32_t *r_len, const int32_t *band,
                              int64_t n_pairs, double *out_score, int32_t *out_end, int n_threads)
{
    struct batch_job job = {q, q_off, q_len, r, r_off, r_len, n_pairs,
                            out_score, NULL, out_end, 0, NULL, band, 0};
    return run_batch(&job, n_threads);
}

int oracle_dtw_band_batch_f32(const float *q, const int64_t *q_off, const int32_t *q_len,
                              const float *r, const int64_t *r_off, const int32_t *r_len, const int32_t *band,
                              int64_t n_pairs, float *out_score, int32_t *out_end, int n_threads)
{
    struct batch_job job = {q, q_off, q_len, r, r_off, r_len, n_pairs,
                            NULL, out_score, out_end, 0, NULL, band, 0};
    return run_batch(&job, n_threads);
}
