/*
 * Plain FP64 CPU oracle for the weighted sort-means (WSM) color quantizer of
 * Celebi, "Fast Color Quantization Using Weighted Sort-Means Clustering".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * GPU library is checked against; it is used by the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark, and by nothing else.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Everything is written for clarity, not speed: `double` arithmetic, no
 * blocking, no reordering, no fused multiply-add (built with
 * -ffp-contract=off).  Each function names the passage of the paper it
 * follows.  Where the paper is silent, the readings used are:
 *   R1  tie rule of the scan: the canonical key (dist, k != p, k) -- on equal
 *       distance keep the previous center p, otherwise the lower index wins.
 *       `literal` = 1 instead applies the printed `dist <= min_dist` test.
 *   R3  memberships start at 0 before the first iteration.
 *   R4  row sort key of M: (d[a][b], b != a, b), so the row's own center is
 *       first even when two centers coincide, and equal distances are ordered
 *       by index.
 *   R5  a center whose cluster is empty keeps its previous value.
 *   R6  SSE_t is the weighted SSE of the assignment made in iteration t
 *       (i.e. of the centers entering iteration t), with weights cnt/N, so it
 *       equals the pixel MSE of those centers.
 *   R7  stop after iteration t when SSE_t == 0, or t >= 2 and
 *       (SSE_{t-1} - SSE_t) / SSE_t <= eps, or t == max_iters.
 *   R13 the palette returned is the one computed by the last update.
 *   R14 pixel mapping uses the key (dist, k != m_i, k) against the final
 *       palette, m_i being the last membership of the pixel's unique color.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "wsm_oracle.h"

#define ORACLE_KEYS (1u << 24)

/* ------------------------------------------------------------------ */
/* Data reduction (Sec. 2, "data sampling"): the unique colors of the image
 * and the number of pixels of each.  The paper finds them with a chained hash
 * table; the set is the same for any hash, and it is emitted here in
 * ascending order of the packed key R<<16 | G<<8 | B, using one counter per
 * possible 24-bit color. */
int64_t oracle_reduce(const uint8_t *rgb, int64_t n_pixels,
                      uint32_t *colors, uint32_t *counts)
{
    if (n_pixels < 0 || n_pixels > (int64_t)UINT32_MAX)
        return -1;
    uint32_t *freq = (uint32_t *)calloc(ORACLE_KEYS, sizeof(uint32_t));
    if (!freq)
        return -2;
    for (int64_t p = 0; p < n_pixels; ++p) {
        uint32_t key = ((uint32_t)rgb[3 * p] << 16) |
                       ((uint32_t)rgb[3 * p + 1] << 8) |
                       (uint32_t)rgb[3 * p + 2];
        freq[key] += 1;
    }
    int64_t n = 0;
    for (uint32_t key = 0; key < ORACLE_KEYS; ++key) {
        if (freq[key] != 0) {
            colors[n] = key;
            counts[n] = freq[key];
            ++n;
        }
    }
    free(freq);
    return n;
}

static void unpack_color(uint32_t key, double x[3])
{
    x[0] = (double)((key >> 16) & 0xFF);
    x[1] = (double)((key >> 8) & 0xFF);
    x[2] = (double)(key & 0xFF);
}

/* Squared Euclidean distance in RGB (Eq. 1 uses ||x - c||_2^2). */
static double sq_dist(const double *a, const double *b)
{
    double d0 = a[0] - b[0];
    double d1 = a[1] - b[1];
    double d2 = a[2] - b[2];
    return d0 * d0 + d1 * d1 + d2 * d2;
}

/* ------------------------------------------------------------------ */
/* Alg. 2, first two steps of the loop body: the pairwise squared distances
 * between centers, d[i][j] = d[j][i] = ||c_i - c_j||^2, and the matrix M whose
 * row i lists all centers in increasing order of distance from c_i (R4). */

typedef struct {
    double d;
    int not_self;
    int idx;
} row_entry;

static int row_entry_cmp(const void *pa, const void *pb)
{
    const row_entry *a = (const row_entry *)pa;
    const row_entry *b = (const row_entry *)pb;
    if (a->d < b->d) return -1;
    if (a->d > b->d) return 1;
    if (a->not_self != b->not_self) return a->not_self - b->not_self;
    return a->idx - b->idx;
}

void oracle_center_tables(const double *c, int K, double *d, int32_t *M)
{
    for (int i = 0; i < K; ++i) {
        d[(size_t)i * K + i] = 0.0;
        for (int j = i + 1; j < K; ++j) {
            double v = sq_dist(&c[3 * i], &c[3 * j]);
            d[(size_t)i * K + j] = v;
            d[(size_t)j * K + i] = v;
        }
    }
    row_entry *row = (row_entry *)malloc(sizeof(row_entry) * (size_t)K);
    for (int i = 0; i < K; ++i) {
        for (int b = 0; b < K; ++b) {
            row[b].d = d[(size_t)i * K + b];
            row[b].not_self = (b != i);
            row[b].idx = b;
        }
        qsort(row, (size_t)K, sizeof(row_entry), row_entry_cmp);
        for (int j = 0; j < K; ++j)
            M[(size_t)i * K + j] = row[j].idx;
    }
    free(row);
}

/* ------------------------------------------------------------------ */
/* Alg. 2, assignment loop (sort-means, Sec. 2 third bullet).  For each point:
 * start from the center p it was assigned to before, prev = min =
 * ||x - c_p||^2; walk M[p] from its second entry; stop as soon as
 * d[p][t] >= 4 prev (then 2 d(x,c_p) <= d(c_p,c_t) for this and every later
 * t, so none of them is closer); otherwise evaluate ||x - c_t||^2 and accept
 * by the tie rule.  `prune` = 0 walks the whole row (full search).
 * Returns the number of point-center distances evaluated, counting the
 * initial ||x - c_p||^2. */
int64_t oracle_search_step(const uint32_t *colors, int64_t n, const double *c,
                           int K, const double *d, const int32_t *M,
                           uint8_t *m, double *min_dist, int prune,
                           int literal)
{
    int64_t evals = 0;
    for (int64_t i = 0; i < n; ++i) {
        double x[3];
        unpack_color(colors[i], x);
        int p = m[i];
        double prev = sq_dist(x, &c[3 * p]);
        double best_d = prev;
        int best = p;
        evals += 1;
        for (int j = 1; j < K; ++j) {
            int t = M[(size_t)p * K + j];
            if (prune && d[(size_t)p * K + t] >= 4.0 * prev)
                break;
            double dist = sq_dist(x, &c[3 * t]);
            evals += 1;
            int accept;
            if (literal)
                accept = (dist <= best_d);
            else
                accept = (dist < best_d) ||
                         (dist == best_d && best != p && t < best);
            if (accept) {
                best_d = dist;
                best = t;
            }
        }
        m[i] = (uint8_t)best;
        if (min_dist)
            min_dist[i] = best_d;
    }
    return evals;
}

/* ------------------------------------------------------------------ */
/* Alg. 2, center update: c_k = (sum_{m[i]=k} w_i x_i) / (sum_{m[i]=k} w_i)
 * with the weights of Sec. 2 ("sample weighting"), w_i = count_i / N.  The
 * factor 1/N is common to the numerator and the denominator, so the center is
 * the count-weighted mean (sum count_i x_i) / (sum count_i).  Both sums are
 * integers below 2^53, exact in double, so the division is the only rounding
 * and the center is the correctly rounded value of the weighted mean.  An
 * empty cluster keeps its center (R5).  `c` is updated in place. */
void oracle_update_step(const uint32_t *colors, const uint32_t *counts,
                        int64_t n, int64_t n_pixels, const uint8_t *m, int K,
                        double *c)
{
    (void)n_pixels;  /* the common factor 1/N of the weights cancels */
    double *sum = (double *)calloc((size_t)K * 4, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        double x[3];
        unpack_color(colors[i], x);
        double w = (double)counts[i];
        int k = m[i];
        sum[4 * k + 0] += w * x[0];
        sum[4 * k + 1] += w * x[1];
        sum[4 * k + 2] += w * x[2];
        sum[4 * k + 3] += w;
    }
    for (int k = 0; k < K; ++k) {
        if (sum[4 * k + 3] > 0.0) {
            c[3 * k + 0] = sum[4 * k + 0] / sum[4 * k + 3];
            c[3 * k + 1] = sum[4 * k + 1] / sum[4 * k + 3];
            c[3 * k + 2] = sum[4 * k + 2] / sum[4 * k + 3];
        }
    }
    free(sum);
}

/* Weighted SSE of one assignment (Eq. 1 with the weights w_i = count_i/N). */
double oracle_weighted_sse(const uint32_t *counts, int64_t n,
                           int64_t n_pixels, const double *min_dist)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += ((double)counts[i] / (double)n_pixels) * min_dist[i];
    return s;
}

/* ------------------------------------------------------------------ */
/* Alg. 2 as a whole, with the termination rules of Sec. 3.2 (fixed number of
 * iterations, or the relative SSE change criterion with threshold eps). */
int oracle_wsm(const uint32_t *colors, const uint32_t *counts, int64_t n,
               int64_t n_pixels, int K, const double *init_centers,
               int max_iters, double eps, int prune, int literal,
               double *centers, uint8_t *m, double *sse_hist,
               int64_t *evals_hist, int32_t *iters_out, int32_t *converged)
{
    if (K < 1 || K > 256 || n < 1 || max_iters < 1)
        return -1;
    double *d = (double *)malloc(sizeof(double) * (size_t)K * K);
    int32_t *M = (int32_t *)malloc(sizeof(int32_t) * (size_t)K * K);
    double *mind = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(centers, init_centers, sizeof(double) * 3 * (size_t)K);
    memset(m, 0, (size_t)n);
    double prev_sse = 0.0;
    int t = 0;
    *converged = 0;
    for (t = 1; t <= max_iters; ++t) {
        oracle_center_tables(centers, K, d, M);
        int64_t ev = oracle_search_step(colors, n, centers, K, d, M, m, mind,
                                        prune, literal);
        double sse = oracle_weighted_sse(counts, n, n_pixels, mind);
        oracle_update_step(colors, counts, n, n_pixels, m, K, centers);
        sse_hist[t - 1] = sse;
        if (evals_hist)
            evals_hist[t - 1] = ev;
        if (sse == 0.0 || (t >= 2 && (prev_sse - sse) / sse <= eps)) {
            *converged = 1;
            break;
        }
        prev_sse = sse;
    }
    *iters_out = (t > max_iters) ? max_iters : t;
    free(d);
    free(M);
    free(mind);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Alg. 1 (conventional batch k-means) on all H*W pixels, full search, with
 * the same tie key as above (previous membership first, then lowest index)
 * and the same termination rules.  Used to check that WSM reaches the same
 * result as plain k-means on the pixels. */
int oracle_kmeans_pixels(const uint8_t *rgb, int64_t n_pixels, int K,
                         const double *init_centers, int max_iters,
                         double eps, double *centers, uint8_t *m,
                         double *sse_hist, int32_t *iters_out,
                         int32_t *converged)
{
    if (K < 1 || K > 256 || n_pixels < 1 || max_iters < 1)
        return -1;
    double *sum = (double *)malloc(sizeof(double) * 4 * (size_t)K);
    memcpy(centers, init_centers, sizeof(double) * 3 * (size_t)K);
    memset(m, 0, (size_t)n_pixels);
    double prev_sse = 0.0;
    int t;
    *converged = 0;
    for (t = 1; t <= max_iters; ++t) {
        double sse = 0.0;
        for (int64_t p = 0; p < n_pixels; ++p) {
            double x[3] = {(double)rgb[3 * p], (double)rgb[3 * p + 1],
                           (double)rgb[3 * p + 2]};
            int mp = m[p];
            int best = -1;
            double best_d = 0.0;
            for (int k = 0; k < K; ++k) {
                double dist = sq_dist(x, &centers[3 * k]);
                int better;
                if (best < 0) {
                    better = 1;
                } else if (dist != best_d) {
                    better = dist < best_d;
                } else if ((k != mp) != (best != mp)) {
                    better = (k == mp);
                } else {
                    better = k < best;
                }
                if (better) {
                    best = k;
                    best_d = dist;
                }
            }
            m[p] = (uint8_t)best;
            sse += best_d;
        }
        sse /= (double)n_pixels;
        memset(sum, 0, sizeof(double) * 4 * (size_t)K);
        for (int64_t p = 0; p < n_pixels; ++p) {
            int k = m[p];
            sum[4 * k + 0] += (double)rgb[3 * p];
            sum[4 * k + 1] += (double)rgb[3 * p + 1];
            sum[4 * k + 2] += (double)rgb[3 * p + 2];
            sum[4 * k + 3] += 1.0;
        }
        for (int k = 0; k < K; ++k) {
            if (sum[4 * k + 3] > 0.0) {
                centers[3 * k + 0] = sum[4 * k + 0] / sum[4 * k + 3];
                centers[3 * k + 1] = sum[4 * k + 1] / sum[4 * k + 3];
                centers[3 * k + 2] = sum[4 * k + 2] / sum[4 * k + 3];
            }
        }
        sse_hist[t - 1] = sse;
        if (sse == 0.0 || (t >= 2 && (prev_sse - sse) / sse <= eps)) {
            *converged = 1;
            break;
        }
        prev_sse = sse;
    }
    *iters_out = (t > max_iters) ? max_iters : t;
    free(sum);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Pixel mapping (Sec. 1, second phase of color quantization) and the MSE of
 * Sec. 3.1: every pixel gets the nearest palette color by the key of R14,
 * searched over all K centers; MSE = (1/HW) sum ||x - x_hat||^2 with the
 * real-valued palette. */

static int64_t find_color(const uint32_t *colors, int64_t n, uint32_t key)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (colors[mid] == key) return mid;
        if (colors[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static int nearest_by_key(const double *x, const double *c, int K, int prefer,
                          double *best_out)
{
    int best = -1;
    double best_d = 0.0;
    for (int k = 0; k < K; ++k) {
        double dist = sq_dist(x, &c[3 * k]);
        int better;
        if (best < 0) better = 1;
        else if (dist != best_d) better = dist < best_d;
        else if ((k != prefer) != (best != prefer)) better = (k == prefer);
        else better = k < best;
        if (better) {
            best = k;
            best_d = dist;
        }
    }
    *best_out = best_d;
    return best;
}

/* Final assignment of every unique color against the final palette.
 * Returns the count-weighted MSE sum_i (count_i/N) * min_i. */
double oracle_assign_colors(const uint32_t *colors, const uint32_t *counts,
                            int64_t n, int64_t n_pixels, const uint8_t *m,
                            const double *c, int K, uint8_t *idx)
{
    double mse = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double x[3], bd;
        unpack_color(colors[i], x);
        idx[i] = (uint8_t)nearest_by_key(x, c, K, m[i], &bd);
        mse += ((double)counts[i] / (double)n_pixels) * bd;
    }
    return mse;
}

int oracle_map(const uint8_t *rgb, int64_t n_pixels, const uint32_t *colors,
               int64_t n_unique, const uint8_t *m, const double *c, int K,
               uint8_t *idx, double *mse_out)
{
    double s = 0.0;
    for (int64_t p = 0; p < n_pixels; ++p) {
        uint32_t key = ((uint32_t)rgb[3 * p] << 16) |
                       ((uint32_t)rgb[3 * p + 1] << 8) |
                       (uint32_t)rgb[3 * p + 2];
        int64_t i = find_color(colors, n_unique, key);
        if (i < 0)
            return -1;
        double x[3] = {(double)rgb[3 * p], (double)rgb[3 * p + 1],
                       (double)rgb[3 * p + 2]};
        double bd;
        idx[p] = (uint8_t)nearest_by_key(x, c, K, m[i], &bd);
        s += bd;
    }
    if (mse_out)
        *mse_out = s / (double)n_pixels;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Differentiable form of the distortion of Eq. 1 (the weighted SSE of a
 * quantization, here over the pixels themselves): with the assignment m
 * frozen,
 *     D(x, c) = (1/N) sum_p ||x_p - c_{m(p)}||^2,
 * a quadratic in the pixel colors x and the palette c, whose derivatives are
 *     dD/dx_p = (2/N) (x_p - c_{m(p)}),
 *     dD/dc_k = (2/N) sum_{p : m(p) = k} (c_k - x_p).
 * x is [n][3] and c [K][3], both double; grad_x and grad_c are scaled by
 * the incoming derivative g = dL/dD. */
double oracle_distortion(const double *x, int64_t n, const uint8_t *m,
                         const double *c, int K)
{
    (void)K;
    double s = 0.0;
    for (int64_t p = 0; p < n; ++p)
        s += sq_dist(&x[3 * p], &c[3 * m[p]]);
    return s / (double)n;
}

void oracle_distortion_grad(const double *x, int64_t n, const uint8_t *m,
                            const double *c, int K, double g,
                            double *grad_x, double *grad_c)
{
    double scale = 2.0 * g / (double)n;
    for (int k = 0; k < 3 * K; ++k)
        grad_c[k] = 0.0;
    for (int64_t p = 0; p < n; ++p) {
        int k = m[p];
        for (int ch = 0; ch < 3; ++ch) {
            double diff = x[3 * p + ch] - c[3 * k + ch];
            grad_x[3 * p + ch] = scale * diff;
            grad_c[3 * k + ch] -= scale * diff;
        }
    }
}
