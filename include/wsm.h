/*
 * wsm.h -- C ABI of the MI355X (gfx950) weighted sort-means color quantizer.
 *
 * The method is the one of M. E. Celebi, "Fast Color Quantization Using
 * Weighted Sort-Means Clustering": batch k-means run on the unique colors of
 * an image (Sec. 2, data sampling), each weighted by its pixel count (Sec. 2,
 * sample weighting), with the sort-means nearest-center search (Sec. 2,
 * third bullet; Alg. 2) and the convergence rule of Sec. 3.2.
 *
 * Conventions for every function below:
 *   - Pointers are DEVICE pointers unless the comment says "host".
 *   - All device work is enqueued asynchronously on `stream`; no function
 *     allocates device memory, frees it, or synchronizes the host, except the
 *     explicit graph handles (wsm_iterate_graph_*), which the caller creates
 *     and destroys.  The library holds no state between calls (apart from
 *     the measurement hook at the end).  Every buffer is owned by the caller
 *     and must stay valid until the enqueued work has finished.
 *   - Return value: WSM_OK (0) or a negative wsm_status.  Arguments are fully
 *     validated on the host before anything is enqueued; on error nothing is
 *     enqueued and no output is written.  WSM_EHIP reports a failed launch.
 *   - Colors are packed keys 0x00RRGGBB (uint32); images are interleaved
 *     8-bit RGB, n_pixels * 3 bytes, any alignment.
 *   - Calls on one stream are ordered; two calls on different streams that
 *     touch the same state or workspace race.
 */
#ifndef WSM_H
#define WSM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WSM_MAX_K 256       /* memberships are stored as uint8 */
#define WSM_HISTORY 1024    /* per-iteration SSE / evaluation records kept */

typedef enum {
    WSM_OK = 0,
    WSM_EINVAL = -1,   /* an argument is out of range or NULL */
    WSM_ENOSPC = -2,   /* workspace, state or output capacity too small */
    WSM_EHIP = -3      /* a HIP launch or device query failed */
} wsm_status;

/* Which points a clustering state holds. */
typedef enum {
    WSM_POINTS_COLORS = 0,  /* unique colors weighted by pixel counts (Alg. 2) */
    WSM_POINTS_PIXELS = 1   /* every pixel with weight 1 (Alg. 1 on the image) */
} wsm_points;

/* Static, never NULL. */
const char *wsm_status_string(int status);

/* ------------------------------------------------------------------ */
/* Data reduction (Sec. 2, "data sampling" and "sample weighting"): the
 * unique colors of an image, in ascending key order, with the number of
 * pixels of each.  The paper uses a hash table; the result is the same set,
 * and this library emits it sorted so that it is reproducible.
 *
 * Host-only size query: bytes of scratch `wsm_reduce_colors` needs for an
 * image of n_pixels.  Returns WSM_EINVAL if n_pixels < 1 or > 2^32 - 1. */
int wsm_reduce_workspace_bytes(int64_t n_pixels, size_t *bytes /* host */);

/* rgb[n_pixels*3] -> colors[cap], counts[cap], *n_unique (device int32).
 * cap must be >= min(n_pixels, 2^24).  workspace: at least
 * wsm_reduce_workspace_bytes(n_pixels) bytes, 16-byte aligned; its contents
 * are scratch.  Entries of colors/counts past *n_unique are left untouched.
 * The sum of counts equals n_pixels. */
int wsm_reduce_colors(const uint8_t *rgb, int64_t n_pixels, uint32_t *colors,
                      uint32_t *counts, int64_t cap, int32_t *n_unique,
                      void *workspace, size_t workspace_bytes,
                      hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * reduction with the library's own workspace, a device array of
 * wsm_reduce_workspace_bytes(WSM_STATIC_MAX_PIXELS) bytes (35.7 MB) that
 * every GPU the library runs on holds until the process ends.  The call
 * itself allocates and frees nothing; its first call on a device (with that
 * device current) looks up the array's address there.  Arguments as for
 * wsm_reduce_colors; n_pixels > WSM_STATIC_MAX_PIXELS returns WSM_ENOSPC.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (on different streams, or from different threads without ordering)
 * race and must not be made; calls ordered on one stream are fine. */
#define WSM_STATIC_MAX_PIXELS (1 << 24)
int wsm_reduce_colors_static(const uint8_t *rgb, int64_t n_pixels,
                             uint32_t *colors, uint32_t *counts, int64_t cap,
                             int32_t *n_unique, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Clustering state.  A caller-owned block of device memory holds the
 * palette, the memberships m[], per-iteration records and scratch; this
 * small host descriptor records its shape so that later calls can size
 * their launches without reading device memory. */
typedef struct wsm_problem {
    int32_t k;            /* number of centers, 1..WSM_MAX_K */
    int32_t points;       /* wsm_points */
    int64_t n_points;     /* unique colors (COLORS) or pixels (PIXELS) */
    int64_t n_pixels;     /* pixels of the image = sum of the weights */
    void *state;          /* device, state_bytes bytes, 256-byte aligned */
    size_t state_bytes;
    const uint32_t *colors; /* COLORS: the table the state is bound to */
    const uint32_t *counts;
    const uint8_t *rgb;     /* PIXELS: the image the state is bound to */
    uint32_t magic;         /* set by wsm_init / wsm_init_pixels */
    int32_t grid;           /* search-kernel blocks, chosen at init (one per
                               compute unit, fewer for small tables); the
                               caller may set any value in 1..2048 before an
                               iterate call, e.g. fewer blocks so that work on
                               other streams gets compute units: memberships,
                               centers, evaluation counts and stopping do not
                               depend on it, the float64 SSE sums only in the
                               order of their terms */
} wsm_problem;

/* Host-only: bytes of state for n_points points and k centers. */
int wsm_state_bytes(int64_t n_points, int k, size_t *bytes /* host */);

/* Initial palette from a subset of the unique colors (Alg. 2 starts from a
 * random subset of the data; the caller draws the indices): palette[3*j..]
 * = (R, G, B) of colors[indices[j]] as float, j < k.  indices: device
 * int32[k], each in [0, n_colors); an index out of range yields (0,0,0) and
 * sets nothing else. */
int wsm_gather_palette(const uint32_t *colors, int64_t n_colors,
                       const int32_t *indices, int k, float *palette,
                       hipStream_t stream);

/* Bind a state to a unique-color table (the output of wsm_reduce_colors,
 * n_unique read back by the caller) and set the initial palette.
 * init_palette: device float[k*3] (R,G,B per center), the random subset of
 * the data that Alg. 2 starts from; copied into the state.  Memberships
 * start at 0 and all records are cleared.  Requires 1 <= k <= min(256,
 * n_unique) and n_pixels = sum(counts) <= 2^32 - 1. */
int wsm_init(wsm_problem *prob /* host, filled */, void *state,
             size_t state_bytes, const uint32_t *colors,
             const uint32_t *counts, int64_t n_unique, int64_t n_pixels,
             int k, const float *init_palette, hipStream_t stream);

/* Same, but the points are the n_pixels pixels of rgb, each of weight 1:
 * Alg. 1 (conventional batch k-means) on the whole image. */
int wsm_init_pixels(wsm_problem *prob /* host, filled */, void *state,
                    size_t state_bytes, const uint8_t *rgb, int64_t n_pixels,
                    int k, const float *init_palette, hipStream_t stream);

/* Run up to max_iters iterations of Alg. 2 (sort-means search + weighted
 * center update).  Iteration t stops the run when SSE_t == 0, or when t >= 2
 * and (SSE_{t-1} - SSE_t) / SSE_t <= eps (Sec. 3.2; eps = 1e-4 in the
 * paper); SSE_t is the weighted SSE of the assignment made in iteration t.
 * A state that has converged stays as it is on further calls; a state that
 * ran out of iterations continues where it stopped.  Requires
 * 1 <= max_iters <= WSM_HISTORY and eps >= 0 and finite. */
int wsm_iterate(const wsm_problem *prob, int max_iters, double eps,
                hipStream_t stream);

/* The same iterations with a full search over all k centers instead of the
 * sort-means scan (plain batch k-means).  With the same initial palette it
 * follows exactly the same trajectory; it is the comparator for timing. */
int wsm_iterate_full(const wsm_problem *prob, int max_iters, double eps,
                     hipStream_t stream);

/* Device pointers into a state.  palette: float4[k] (R,G,B,0) after the
 * last update; palette64: the same centers in float64, double4[k] (R,G,B,0)
 * -- each the correctly rounded count-weighted mean of its cluster (Alg. 2,
 * last loop), of which palette is the float32 rounding; the searches choose
 * centers as float64 arithmetic on palette64 does, with ties kept by the
 * previous center, then the lower index; membership: uint8[n_points];
 * sse_history / evals_history:
 * [WSM_HISTORY], entry t-1 for iteration t (SSE_t normalised by n_pixels,
 * i.e. the MSE of the palette entering iteration t; evals = the distance
 * evaluations of Alg. 2's scan, summed over the points: 1 + the centers
 * before the break per point for wsm_iterate, k per point for
 * wsm_iterate_full); info: int32[4] = {iterations done, converged,
 * device error flags, reserved}. */
typedef struct wsm_views {
    const float *palette;
    const uint8_t *membership;
    const double *sse_history;
    const int64_t *evals_history;
    const int32_t *info;
    const double *palette64;
} wsm_views;
int wsm_state_views(const wsm_problem *prob, wsm_views *views /* host */);

/* ------------------------------------------------------------------ */
/* Pixel mapping (Sec. 1, second phase of color quantization): assign every
 * pixel of rgb to its nearest palette color.  Each unique color is first
 * assigned by a sort-means scan against the final palette starting from its
 * last membership (ties keep that membership, then the lower index); the
 * result is scattered into lut (device uint8[2^24], scratch, only entries of
 * colors present in the table are written or read) and gathered per pixel
 * into index_out[n_pixels].  Optional outputs (pass NULL to skip):
 * rgb_out[n_pixels*3] with the palette rounded half-to-even and clamped to
 * 0..255, and mse_out[1] (device double) = (1/N) sum ||x - c_idx||^2 with the
 * real-valued palette (Sec. 3.1).  Requires a COLORS state and an image
 * whose colors are all in the state's table (the image it was reduced from).
 */
int wsm_map_pixels(const wsm_problem *prob, const uint8_t *rgb,
                   int64_t n_pixels, uint8_t *lut, uint8_t *index_out,
                   uint8_t *rgb_out, double *mse_out, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Batched persistent form: the iterations of many images (their own
 * tables, K, iteration budgets and eps), each bound to its own state by
 * wsm_init, run by one launch of persistent blocks that take work items
 * from a device queue -- per image and step, the update with the row sort
 * of M (in parts of rows_per_item rows) and the sort-means search (in grid
 * virtual blocks).  Each image's result is that of wsm_iterate(max_iters,
 * eps) on it, bit for bit.
 *   probs[n_images] (host): initialised COLORS problems on one device, with
 *     255 * n_pixels < 2^32; at most 128 images.
 *   max_iters, eps (host, per image): as for wsm_iterate.
 *   grid, rows_per_item (host, per image, nullable; 0 = default): the work
 *     split (search blocks, 1..2048, default the problem's grid; rows per
 *     rows item, default 1), as an autotuner picks them.
 * wsm_batch_create binds a caller-owned workspace (256-byte aligned, at
 * least wsm_batch_workspace_bytes) and records the queue reset and the
 * persistent launch into a HIP graph; it synchronizes the host once (set-up
 * copies) and the runtime may reserve device memory for the graph.
 * wsm_batch_launch enqueues a whole run on `stream`; states must have been
 * re-initialised (wsm_init) if they should start over.  wsm_batch_error
 * gives a device int32 with error bits of the last run (1: a block gave up
 * waiting, 2: the queue overflowed; 0 when all is well).  Launches of one
 * handle must not overlap. */
typedef struct wsm_batch wsm_batch;
int wsm_batch_workspace_bytes(int n_images, const wsm_problem *probs,
                              const int32_t *max_iters, const int32_t *grid,
                              const int32_t *rows_per_item, size_t *bytes /* host */);
int wsm_batch_create(int n_images, const wsm_problem *probs, const int32_t *max_iters,
                     const double *eps, const int32_t *grid,
                     const int32_t *rows_per_item, void *workspace,
                     size_t workspace_bytes, wsm_batch **batch /* host, out */);
int wsm_batch_launch(wsm_batch *batch, hipStream_t stream);
int wsm_batch_error(const wsm_batch *batch, const int32_t **err /* host, out */);
int wsm_batch_destroy(wsm_batch *batch);

/* ------------------------------------------------------------------ */
/* Differentiable form (for training systems; the quantization itself is
 * not differentiated).  The distortion of Eq. 1, taken over the pixels with
 * the assignment m frozen (the pixel map's indices), for a batch of images:
 *     D_i = (1/N) sum_p ||x_ip - c_{i,m(p)}||^2,
 * and its adjoint dD/dx_ip = (2/N)(x_ip - c_{i,m(p)}) and
 * dD/dc_ik = (2/N) sum_{m(p)=k} (c_ik - x_ip).  D is piecewise quadratic;
 * away from assignment ties these are its derivatives.
 *   x:       float [batch][n_pixels][3], pixel colors (any real values)
 *   index:   uint8 [batch][n_pixels], each < k (larger values read an
 *            unspecified palette slot, never memory outside the call)
 *   palette: float [batch][k][3]
 * Sums are taken in float64; block partials go to workspace (at least
 * wsm_distortion_workspace_bytes, 16-byte aligned) and are added in a fixed
 * order.  x, palette and the float outputs must be 4-byte aligned. */
int wsm_distortion_workspace_bytes(int batch, int64_t n_pixels, int k,
                                   size_t *bytes /* host */);
/* d_out: device double [batch]. */
int wsm_distortion(const float *x, const uint8_t *index, const float *palette,
                   int batch, int64_t n_pixels, int k, double *d_out,
                   void *workspace, size_t workspace_bytes, hipStream_t stream);
/* grad_d: device double [batch], dL/dD_i.  grad_x (float [batch][n][3]) and
 * grad_palette (float [batch][k][3]) are written when not NULL (at least
 * one must be given). */
int wsm_distortion_backward(const float *x, const uint8_t *index,
                            const float *palette, int batch, int64_t n_pixels,
                            int k, const double *grad_d, float *grad_x,
                            float *grad_palette, void *workspace,
                            size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Launch replay (not part of the method).  wsm_iterate and
 * wsm_iterate_full enqueue a fixed sequence of kernel launches that depends
 * only on their arguments, and they can be captured into a HIP graph by the
 * caller like any stream work.  These calls do that for the caller, with an
 * opaque handle the caller owns:
 *   - create records the sequence of wsm_iterate (full = 0) or
 *     wsm_iterate_full (full != 0) for prob, max_iters and eps into a graph,
 *     on a stream of its own that it destroys again, and instantiates it
 *     (host work of a few milliseconds; the runtime may reserve device
 *     memory for the graph).  Nothing runs on the device.  Validation as for
 *     wsm_iterate; *graph is NULL on error.
 *   - launch enqueues the whole sequence on `stream`; the effect is that of
 *     the corresponding iterate call with the same arguments.  The state,
 *     points and prob's buffers must be the ones the graph was created for
 *     (re-initialising the same state with wsm_init is allowed).
 *   - destroy releases the graph; the caller must not launch it afterwards.
 *     Work already enqueued is not affected.
 * A handle may be launched from any thread, but not by two threads at once. */
typedef struct wsm_graph wsm_graph;
int wsm_iterate_graph_create(const wsm_problem *prob, int max_iters, double eps,
                             int full, wsm_graph **graph /* host, out */);
int wsm_iterate_graph_launch(wsm_graph *graph, hipStream_t stream);
int wsm_iterate_graph_destroy(wsm_graph *graph);

/* ------------------------------------------------------------------ */
/* Measurement support (not part of the method).  While attached, every
 * launch of the kernel `which` made by this process is made with
 * hipExtLaunchKernelGGL and two HIP events, which the runtime records when
 * the kernel starts and when it ends, on the stream it is launched on;
 * wsm_timing_read waits for them and returns the first min(count, capacity)
 * durations in ms.  The hook is process-wide: its calls and the launches it
 * claims events for take one lock, so they may come from several threads,
 * but detach must not run while another thread launches the timed kernel
 * (that launch may still be using the events it claimed).  Attach creates
 * 2 * capacity events and detach destroys them.  Attaching while attached
 * returns WSM_EINVAL. */
typedef enum {
    WSM_KERNEL_REDUCE_PARTITION = 1,
    WSM_KERNEL_REDUCE_COMPACT = 2,
    WSM_KERNEL_ROWS = 3,
    WSM_KERNEL_SEARCH = 4,
    WSM_KERNEL_MAP_ASSIGN = 5,
    WSM_KERNEL_MAP_GATHER = 6,
    WSM_KERNEL_FULL_STEP = 7
} wsm_kernel;
int wsm_timing_attach(int which, int capacity);
int wsm_timing_read(float *ms /* host [capacity] */, int capacity,
                    int *count /* host */);
int wsm_timing_detach(void);

#ifdef __cplusplus
}
#endif

#endif /* WSM_H */
