/*
 * FP64 CPU oracle of the weighted sort-means color quantizer.
 * TEST INFRASTRUCTURE ONLY: see wsm_oracle.c for the readings it implements.
 */
#ifndef WSM_ORACLE_H
#define WSM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Unique colors, ascending packed 0x00RRGGBB, with pixel counts.  Returns
 * the number of unique colors, or < 0 on error. */
int64_t oracle_reduce(const uint8_t *rgb, int64_t n_pixels,
                      uint32_t *colors, uint32_t *counts);

/* d[K*K] squared center distances and M[K*K] sorted neighbour rows. */
void oracle_center_tables(const double *c, int K, double *d, int32_t *M);

/* One assignment pass; m is read (previous) and written (new). */
int64_t oracle_search_step(const uint32_t *colors, int64_t n, const double *c,
                           int K, const double *d, const int32_t *M,
                           uint8_t *m, double *min_dist, int prune,
                           int literal);

/* One weighted centroid update; c[K*3] is updated in place. */
void oracle_update_step(const uint32_t *colors, const uint32_t *counts,
                        int64_t n, int64_t n_pixels, const uint8_t *m, int K,
                        double *c);

double oracle_weighted_sse(const uint32_t *counts, int64_t n,
                           int64_t n_pixels, const double *min_dist);

/* Full WSM run from init_centers[K*3]. */
int oracle_wsm(const uint32_t *colors, const uint32_t *counts, int64_t n,
               int64_t n_pixels, int K, const double *init_centers,
               int max_iters, double eps, int prune, int literal,
               double *centers, uint8_t *m, double *sse_hist,
               int64_t *evals_hist, int32_t *iters_out, int32_t *converged);

/* Alg. 1 on all pixels (full search). */
int oracle_kmeans_pixels(const uint8_t *rgb, int64_t n_pixels, int K,
                         const double *init_centers, int max_iters,
                         double eps, double *centers, uint8_t *m,
                         double *sse_hist, int32_t *iters_out,
                         int32_t *converged);

/* Final assignment of the unique colors; returns the weighted MSE. */
double oracle_assign_colors(const uint32_t *colors, const uint32_t *counts,
                            int64_t n, int64_t n_pixels, const uint8_t *m,
                            const double *c, int K, uint8_t *idx);

/* Per-pixel palette index and MSE. */
int oracle_map(const uint8_t *rgb, int64_t n_pixels, const uint32_t *colors,
               int64_t n_unique, const uint8_t *m, const double *c, int K,
               uint8_t *idx, double *mse_out);

/* Distortion of Eq. 1 over pixels x[n][3] with frozen assignment m, and its
 * gradients (scaled by g) with respect to x and the palette c[K][3]. */
double oracle_distortion(const double *x, int64_t n, const uint8_t *m,
                         const double *c, int K);
void oracle_distortion_grad(const double *x, int64_t n, const uint8_t *m,
                            const double *c, int K, double g,
                            double *grad_x, double *grad_c);

#ifdef __cplusplus
}
#endif

#endif
