// Iterations of the weighted sort-means loop (Alg. 2) on gfx950: two
// launches per iteration for K > kFusedMaxK, one for smaller K (the fused
// kernel sorts the rows inside every search block) and for the full-search
// comparator.
//
// Step i, rows launch (one block per center p):
//   1. every block applies the center update of step i-1 (Alg. 2, last
//      loop: c_k = sum w x / sum w, from exact integer sums of
//      count * channel), reduces the SSE partials of step i-1 in a fixed
//      order and evaluates the Sec. 3.2 stopping rule -- redundantly, so all
//      blocks agree without a grid-wide barrier; block 0 publishes the
//      palette and the record;
//   2. block p sorts row p of the neighbour matrix M for the new centers
//      (Sec. 2: the inter-center distances with every row sorted).
// Step i, search launch (each block takes the 64-color chunks b, b + grid,
// ...; its waves take them one at a time from an LDS counter):
//   3. sort-means from each point's previous center over an LDS copy of M
//      (the launch variants kVar* of sm_block.h: after a call's first step,
//      each lane scans the first entries of its point's row, a wave's
//      further scans over the row heads are spread over its lanes and the
//      rare longer ones finished by whole waves);
//   4. sums count * (R, G, B, 1) per center: runs of equal centers within a
//      wave are pre-summed with a segmented scan, then added into LDS, and
//      each block flushes its non-zero sums with 64-bit device atomics into
//      its XCD's copy of the totals (the second level of the reduction);
//      the block's SSE and evaluation count go to per-block partials.
// The full-search comparator does 1, 3 (full search) and 4 in one launch.
// The sums are exact integers, so the result does not depend on the order
// of the additions and the pruned search, the full search and k-means on the
// raw pixels produce bit-identical centers.
//
// Records and palettes are double-buffered by step parity and the totals
// triple-buffered, so no launch reads what another block of the same launch
// writes.  A single-block kernel applies the final update after the last
// step and copies the result to the public slot 0.
#include <new>

#include "iter_device.h"

namespace wsm {

// Sort-means step i, first launch: the update of step i-1 in every block
// (see the file comment), then block p sorts row p of M for the new
// centers.  Block 0 clears the totals slot step i accumulates into.
template <bool PACKED>
__global__ __launch_bounds__(kSortThreads) void rows_kernel(IterArgs a, int i) {
    __shared__ RowsLds L;
    rows_body<PACKED>(a, i, blockIdx.x, blockIdx.x + 1, L);
}

// Sort-means step i, second launch: every block copies the centers and M
// into LDS and searches its chunk.
template <bool PACKED, int V>
__global__ __launch_bounds__(kSearchThreads) void search_kernel(IterArgs a, int i) {
    __shared__ SearchLds<V> L;
    search_body<PACKED, V>(a, i, blockIdx.x, L);
}

// Rows of M for palette slot 0 of the state (the pixel map's palette).
__global__ __launch_bounds__(kSortThreads) void palette_rows_kernel(StateView sv, int K) {
    __shared__ float4 cen[kMaxK];
    __shared__ __align__(16) unsigned long long keys[kMaxK];
    __shared__ uint32_t rank[kMaxK];
    for (int c = threadIdx.x; c < K; c += kSortThreads) cen[c] = sv.pal[c];
    sort_row<kSortThreads>(cen, K, blockIdx.x, keys, rank, sv.rows + (size_t)blockIdx.x * kRowStride,
                           sv.rowd + (size_t)blockIdx.x * kRowDist);
}

// Sort-means step for K <= kFusedMaxK in one launch: every block applies
// the update as in the rows launch, sorts all K rows of M into LDS itself
// (thread (p, t) ranks center t in row p, and also writes the row table
// entry) and searches its points.  Totals slots follow the comparator's
// order: clear (i + 1) % 3, add into i % 3.
template <bool PACKED>
__global__ __launch_bounds__(kSearchThreads) void fused_step_kernel(IterArgs a, int i) {
    __shared__ float4 cen[kMaxK];
    __shared__ double4 cen64[kMaxK];
    __shared__ unsigned long long acc[kMaxK * 4];
    __shared__ __align__(16) unsigned long long keys[kFusedMaxK * kFusedMaxK];
    __shared__ __align__(16) uint8_t Ms[kFusedMaxK * kFusedMaxK];
    __shared__ float4 Tb[kFusedMaxK * kFusedMaxK];
    __shared__ double dscr[kSearchThreads / 64];
    __shared__ unsigned long long uscr[kSearchThreads / 64];
    __shared__ uint32_t next;
    constexpr int NT = kSearchThreads;
    constexpr int NACC = PACKED ? 2 : 4;
    static_assert(kFusedMaxK * kFusedMaxK <= NT, "one thread per row entry");
    const int tid = threadIdx.x;
    const int K = a.k;
    uint32_t key[kCpt], cnt[kCpt];
    int pm[kCpt];
    prefetch_points(a, blockIdx.x, key, cnt, pm);
    const Record rec = update_phase<NT, PACKED>(a, i, cen, cen64, blockIdx.x == 0, dscr, uscr, acc);
    if (rec.converged) return;
    if (blockIdx.x == 0) {
        clear_totals<NT, PACKED>(a.sv.totals + (size_t)((i + 1) % 3) * kTotSlot, a.k);
    }
    for (int c = tid; c < K * NACC; c += NT) acc[c] = 0ull;
    const int p = tid / kFusedMaxK, t = tid % kFusedMaxK;
    const bool entry = p < K && t < K && t != p;
    unsigned long long kt = ~0ull;
    float4 ct = make_float4(0.f, 0.f, 0.f, 0.f);
    if (entry) {
        const float4 cp = cen[p];
        ct = cen[t];
        kt = ((unsigned long long)__float_as_uint(sq_dist(cp.x, cp.y, cp.z, ct.x, ct.y, ct.z))
              << 32) | (unsigned)t;
    }
    keys[tid] = kt;
    if (tid == 0) next = 0u;
    __syncthreads();
    if (entry) {
        const ulonglong2 *k2 = (const ulonglong2 *)(keys + p * kFusedMaxK);
        uint32_t r = 0;
#pragma unroll
        for (int u = 0; u < kFusedMaxK / 2; ++u) {
            const ulonglong2 v = k2[u];
            r += (uint32_t)(v.x < kt) + (uint32_t)(v.y < kt);
        }
        Ms[p * lds_row_stride(K) + r] = (uint8_t)t;
        Tb[p * kFusedMaxK + r] = make_float4(ct.x, ct.y, ct.z, __uint_as_float((uint32_t)(kt >> 32)));
    }
    __syncthreads();
    // a fresh state (no step completed) starts from center 0 everywhere:
    // the full scan gives the same centers (see search_chunk)
    search_chunk<PACKED, false, false, true>(a, i, blockIdx.x, rec.mode, cen, cen64, Ms, acc, dscr,
                                             uscr, nullptr, &next, key, cnt, pm, rec.iters == 0,
                                             nullptr, nullptr, Tb, kFusedMaxK);
}

// Full-search comparator: one launch per step, the update applied
// redundantly by every block as in the sort-means step.
template <bool PACKED>
__global__ __launch_bounds__(kSearchThreads) void full_step_kernel(IterArgs a, int i) {
    __shared__ float4 cen[kMaxK];
    __shared__ double4 cen64[kMaxK];
    __shared__ unsigned long long acc[kMaxK * 4];
    __shared__ double dscr[kSearchThreads / 64];
    __shared__ unsigned long long uscr[kSearchThreads / 64];
    __shared__ uint32_t next;
    constexpr int NT = kSearchThreads;
    constexpr int NACC = PACKED ? 2 : 4;
    const int tid = threadIdx.x;
    uint32_t key[kCpt], cnt[kCpt];
    int pm[kCpt];
    prefetch_points(a, blockIdx.x, key, cnt, pm);
    const Record rec = update_phase<NT, PACKED>(a, i, cen, cen64, blockIdx.x == 0, dscr, uscr, acc);
    if (rec.converged) return;
    if (blockIdx.x == 0) {
        clear_totals<NT, PACKED>(a.sv.totals + (size_t)((i + 1) % 3) * kTotSlot, a.k);
    }
    for (int c = tid; c < a.k * NACC; c += NT) acc[c] = 0ull;
    if (tid == 0) next = 0u;
    __syncthreads();
    search_chunk<PACKED, true, false>(a, i, blockIdx.x, rec.mode, cen, cen64, nullptr, acc, dscr,
                                      uscr, nullptr, &next, key, cnt, pm);
}

// Final update after the last step of a call (one block).  Publishes the
// palette and record to slot 0 and clears totals[0] for the next call.
template <bool PACKED>
__global__ __launch_bounds__(kRowThreads) void final_kernel(IterArgs a, int i) {
    __shared__ FinalLds<kRowThreads> L;
    final_body<kRowThreads, PACKED>(a, i, L);
}

// State initialisation: header, palette slot 0, cleared records, totals,
// histories and memberships.
__global__ void init_state_kernel(StateView sv, int k, int points, int grid,
                                  int64_t n_points, int64_t n_pixels,
                                  const float *__restrict__ init_palette) {
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (blockIdx.x == 0) {
        // the palette's flags, its centers spread over the first block
        int flags = 0;
        for (int c = threadIdx.x; c < k; c += blockDim.x)
            flags |= center_flags(make_double4((double)init_palette[3 * c],
                                               (double)init_palette[3 * c + 1],
                                               (double)init_palette[3 * c + 2], 0.0));
        flags = __syncthreads_or(flags & kFlagWild);
        if (threadIdx.x == 0) {
            Header *h = sv.hdr;
            h->magic = kMagic;
            h->k = k;
            h->points = points;
            h->grid = grid;
            h->n_points = n_points;
            h->n_pixels = n_pixels;
            h->wild = flags ? 1 : 0;
            h->pad = 0;
            for (int j = 0; j < 3; ++j) h->reserved[j] = 0ull;
            Record z;
            z.iters = 0;
            z.converged = 0;
            z.err = 0;
            z.mode = kModeResolve;
            z.sse_last = 0.0;
            z.pad2 = 0.0;
            h->rec[0] = z;
            h->rec[1] = z;
            for (int j = 0; j < 4; ++j) h->info[j] = 0;
        }
    }
    for (int64_t c = gt; c < 2 * kMaxK; c += stride) {
        const int64_t j = c % kMaxK;  // both slots hold the initial palette
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j < k) v = make_float4(init_palette[3 * j], init_palette[3 * j + 1],
                                   init_palette[3 * j + 2], 0.f);
        sv.pal[c] = v;
        sv.pal64[c] = make_double4((double)v.x, (double)v.y, (double)v.z, 0.0);
    }
    for (int64_t c = gt; c < 3 * (int64_t)kTotSlot; c += stride) sv.totals[c] = 0ull;
    for (int64_t c = gt; c < 2 * kMaxGrid; c += stride) {
        sv.sse_part[c] = 0.0;
        sv.eval_part[c] = 0ull;
    }
    for (int64_t c = gt; c < kHistory; c += stride) {
        sv.sse_hist[c] = 0.0;
        sv.eval_hist[c] = 0ll;
    }
    for (int64_t c = gt; c < n_points; c += stride) sv.m[c] = 0;
}

// Initial palette from indices into the unique-color table.
__global__ void gather_palette_kernel(const uint32_t *__restrict__ colors, int64_t n,
                                      const int32_t *__restrict__ idx, int k,
                                      float *__restrict__ pal) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    const int32_t i = idx[j];
    float r = 0.f, g = 0.f, b = 0.f;
    if (i >= 0 && (int64_t)i < n) unpack_key(colors[i], r, g, b);
    pal[3 * j + 0] = r;
    pal[3 * j + 1] = g;
    pal[3 * j + 2] = b;
}

}  // namespace wsm

using namespace wsm;

// ---------------------------------------------------------------------------
// Host side.

static int device_cus(int *cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return WSM_EHIP;
    if (hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return WSM_EHIP;
    if (*cus < 1) *cus = 1;
    return WSM_OK;
}

extern "C" int wsm_state_bytes(int64_t n_points, int k, size_t *bytes) {
    if (!bytes || n_points < 1 || n_points > (int64_t)0xFFFFFFFFll || k < 1 || k > kMaxK)
        return WSM_EINVAL;
    *bytes = state_bytes_for(n_points);
    return WSM_OK;
}

static int init_common(wsm_problem *prob, void *state, size_t state_bytes, int points,
                       const uint32_t *colors, const uint32_t *counts, const uint8_t *rgb,
                       int64_t n_points, int64_t n_pixels, int k, const float *init_palette,
                       hipStream_t stream) {
    if (!prob || !state || !init_palette) return WSM_EINVAL;
    if (k < 1 || k > kMaxK || n_points < 1 || k > n_points) return WSM_EINVAL;
    if (n_pixels < 1 || n_pixels > (int64_t)0xFFFFFFFFll) return WSM_EINVAL;
    if (((uintptr_t)state & 255u) != 0u) return WSM_EINVAL;
    if (state_bytes < state_bytes_for(n_points)) return WSM_ENOSPC;
    int cus = 0;
    int rc = device_cus(&cus);
    if (rc != WSM_OK) return rc;
    // One block per CU, fewer for small tables (at least 256 points per
    // block), more when a block would otherwise need more than two passes.
    int64_t grid = cus;
    const int64_t by_size = (n_points + 255) / 256;
    if (by_size < grid) grid = by_size;
    const int64_t by_pass = (n_points + 2 * (int64_t)kPass - 1) / (2 * (int64_t)kPass);
    if (by_pass > grid) grid = by_pass;
    if (grid > kMaxGrid) grid = kMaxGrid;
    if (grid < 1) grid = 1;
    StateView sv = make_view(state);
    (void)hipGetLastError();
    init_state_kernel<<<dim3(256), dim3(256), 0, stream>>>(sv, k, points, (int)grid, n_points,
                                                          n_pixels, init_palette);
    if (hipGetLastError() != hipSuccess) return WSM_EHIP;
    prob->k = k;
    prob->points = points;
    prob->n_points = n_points;
    prob->n_pixels = n_pixels;
    prob->state = state;
    prob->state_bytes = state_bytes;
    prob->colors = colors;
    prob->counts = counts;
    prob->rgb = rgb;
    prob->magic = kMagic;
    prob->grid = (int)grid;
    return WSM_OK;
}

extern "C" int wsm_init(wsm_problem *prob, void *state, size_t state_bytes,
                        const uint32_t *colors, const uint32_t *counts, int64_t n_unique,
                        int64_t n_pixels, int k, const float *init_palette,
                        hipStream_t stream) {
    if (!colors || !counts) return WSM_EINVAL;
    if (n_unique > (1ll << 24) || n_unique > n_pixels) return WSM_EINVAL;
    return init_common(prob, state, state_bytes, WSM_POINTS_COLORS, colors, counts, nullptr,
                       n_unique, n_pixels, k, init_palette, stream);
}

extern "C" int wsm_init_pixels(wsm_problem *prob, void *state, size_t state_bytes,
                               const uint8_t *rgb, int64_t n_pixels, int k,
                               const float *init_palette, hipStream_t stream) {
    if (!rgb) return WSM_EINVAL;
    return init_common(prob, state, state_bytes, WSM_POINTS_PIXELS, nullptr, nullptr, rgb,
                       n_pixels, n_pixels, k, init_palette, stream);
}

static int check_problem(const wsm_problem *prob) {
    if (!prob || prob->magic != kMagic || !prob->state) return WSM_EINVAL;
    if (prob->k < 1 || prob->k > kMaxK || prob->n_points < 1) return WSM_EINVAL;
    if (prob->grid < 1 || prob->grid > kMaxGrid) return WSM_EINVAL;
    if (prob->n_pixels < 1 || prob->n_pixels > (int64_t)0xFFFFFFFFll) return WSM_EINVAL;
    if (prob->points == WSM_POINTS_COLORS) {
        if (!prob->colors || !prob->counts) return WSM_EINVAL;
    } else if (prob->points == WSM_POINTS_PIXELS) {
        if (!prob->rgb) return WSM_EINVAL;
    } else {
        return WSM_EINVAL;
    }
    if (prob->state_bytes < state_bytes_for(prob->n_points)) return WSM_ENOSPC;
    return WSM_OK;
}

int wsm_internal_check_problem(const wsm_problem *prob) { return check_problem(prob); }

static IterArgs make_args(const wsm_problem *prob, double eps) {
    IterArgs a;
    a.sv = make_view(prob->state);
    a.pts.colors = prob->colors;
    a.pts.counts = prob->counts;
    a.pts.rgb = prob->rgb;
    a.pts.n = prob->n_points;
    a.pts.is_pixels = prob->points == WSM_POINTS_PIXELS ? 1 : 0;
    a.k = prob->k;
    a.grid = prob->grid;
    a.n_pixels = prob->n_pixels;
    a.eps = eps;
    return a;
}

static int check_iter_args(const wsm_problem *prob, int max_iters, double eps) {
    int rc = check_problem(prob);
    if (rc != WSM_OK) return rc;
    if (max_iters < 1 || max_iters > kHistory) return WSM_EINVAL;
    if (!(eps >= 0.0) || eps > 1e300) return WSM_EINVAL;  // rejects NaN and inf
    return WSM_OK;
}

// Exact packing of the four sums into two 64-bit words needs 255 N < 2^32.
static bool packed_sums(const wsm_problem *prob) {
    return (unsigned long long)prob->n_pixels * 255ull < (1ull << 32);
}

template <bool PACKED>
static int launch_steps(const IterArgs &a, int max_iters, bool full, hipStream_t stream) {
    for (int i = 0; i < max_iters; ++i) {
        if (full) {
            WSM_LAUNCH(WSM_KERNEL_FULL_STEP, full_step_kernel<PACKED>, dim3(a.grid),
                       dim3(kSearchThreads), stream, a, i);
        } else if (a.k <= kFusedMaxK) {
            WSM_LAUNCH(WSM_KERNEL_SEARCH, fused_step_kernel<PACKED>, dim3(a.grid),
                       dim3(kSearchThreads), stream, a, i);
        } else {
            WSM_LAUNCH(WSM_KERNEL_ROWS, rows_kernel<PACKED>, dim3(a.k), dim3(kSortThreads), stream,
                       a, i);
            // K >= kDeferMinK here
            const auto search =
                i == 0 ? search_kernel<PACKED, kVarFirst> : search_kernel<PACKED, kVarDefer>;
            WSM_LAUNCH(WSM_KERNEL_SEARCH, search, dim3(a.grid), dim3(kSearchThreads), stream, a,
                       i);
        }
    }
    final_kernel<PACKED><<<dim3(1), dim3(kRowThreads), 0, stream>>>(a, max_iters);
    return hipGetLastError() == hipSuccess ? WSM_OK : WSM_EHIP;
}

// Rows of M for the state's published palette (used by the pixel map).
int wsm_internal_palette_rows(void *state, int k, hipStream_t stream) {
    palette_rows_kernel<<<dim3(k), dim3(kSortThreads), 0, stream>>>(make_view(state), k);
    return hipGetLastError() == hipSuccess ? WSM_OK : WSM_EHIP;
}

static int launch_direct(const IterArgs &a, int max_iters, bool full, bool packed,
                         hipStream_t stream) {
    return packed ? launch_steps<true>(a, max_iters, full, stream)
                  : launch_steps<false>(a, max_iters, full, stream);
}

static int iterate_impl(const wsm_problem *prob, int max_iters, double eps, bool full,
                        hipStream_t stream) {
    int rc = check_iter_args(prob, max_iters, eps);
    if (rc != WSM_OK) return rc;
    const IterArgs a = make_args(prob, eps);
    (void)hipGetLastError();
    return launch_direct(a, max_iters, full, packed_sums(prob), stream);
}

// ---------------------------------------------------------------------------
// A caller-owned HIP graph of one call's launch sequence.  The sequence
// depends only on the call's arguments, so it is recorded once (on a stream
// the create call makes and destroys) and replayed by every launch.
struct wsm_graph {
    uint32_t magic;
    hipGraphExec_t exec;
};

constexpr uint32_t kGraphMagic = 0x574D4752u;

extern "C" int wsm_iterate_graph_create(const wsm_problem *prob, int max_iters, double eps,
                                        int full, wsm_graph **graph) {
    if (!graph) return WSM_EINVAL;
    *graph = nullptr;
    int rc = check_iter_args(prob, max_iters, eps);
    if (rc != WSM_OK) return rc;
    const IterArgs a = make_args(prob, eps);
    (void)hipGetLastError();
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return WSM_EHIP;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    rc = WSM_EHIP;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        const int lrc = launch_direct(a, max_iters, full != 0, packed_sums(prob), cs);
        const hipError_t end = hipStreamEndCapture(cs, &g);
        if (lrc == WSM_OK && end == hipSuccess && g &&
            hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess)
            rc = WSM_OK;
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    (void)hipGetLastError();
    if (rc != WSM_OK) return rc;
    wsm_graph *h = new (std::nothrow) wsm_graph;
    if (!h) {
        (void)hipGraphExecDestroy(exec);
        return WSM_EHIP;
    }
    h->magic = kGraphMagic;
    h->exec = exec;
    *graph = h;
    return WSM_OK;
}

extern "C" int wsm_iterate_graph_launch(wsm_graph *graph, hipStream_t stream) {
    if (!graph || graph->magic != kGraphMagic) return WSM_EINVAL;
    return hipGraphLaunch(graph->exec, stream) == hipSuccess ? WSM_OK : WSM_EHIP;
}

extern "C" int wsm_iterate_graph_destroy(wsm_graph *graph) {
    if (!graph) return WSM_OK;
    if (graph->magic != kGraphMagic) return WSM_EINVAL;
    const hipError_t e = hipGraphExecDestroy(graph->exec);
    graph->magic = 0u;
    delete graph;
    return e == hipSuccess ? WSM_OK : WSM_EHIP;
}

extern "C" int wsm_iterate(const wsm_problem *prob, int max_iters, double eps,
                           hipStream_t stream) {
    return iterate_impl(prob, max_iters, eps, false, stream);
}

extern "C" int wsm_iterate_full(const wsm_problem *prob, int max_iters, double eps,
                                hipStream_t stream) {
    return iterate_impl(prob, max_iters, eps, true, stream);
}

extern "C" int wsm_state_views(const wsm_problem *prob, wsm_views *views) {
    if (!views) return WSM_EINVAL;
    int rc = check_problem(prob);
    if (rc != WSM_OK) return rc;
    const StateView sv = make_view(prob->state);
    views->palette = (const float *)sv.pal;
    views->palette64 = (const double *)sv.pal64;
    views->membership = sv.m;
    views->sse_history = sv.sse_hist;
    views->evals_history = (const int64_t *)sv.eval_hist;
    views->info = sv.hdr->info;
    return WSM_OK;
}

extern "C" int wsm_gather_palette(const uint32_t *colors, int64_t n_colors,
                                  const int32_t *indices, int k, float *palette,
                                  hipStream_t stream) {
    if (!colors || !indices || !palette || n_colors < 1 || k < 1 || k > kMaxK) return WSM_EINVAL;
    (void)hipGetLastError();
    gather_palette_kernel<<<dim3(1), dim3(kMaxK), 0, stream>>>(colors, n_colors, indices, k,
                                                               palette);
    return hipGetLastError() == hipSuccess ? WSM_OK : WSM_EHIP;
}
