// Iterations of the weighted sort-means loop (Alg. 2) on gfx950.
//
// One iteration t = call-relative step i is two launches:
//   rows    K blocks.  Every block applies the weighted center update of the
//           previous step (Alg. 2, last loop: c_k = sum w x / sum w, here
//           with exact integer sums of count * channel), evaluates the Sec.
//           3.2 stopping rule, and then builds row a = blockIdx of the
//           sorted-neighbour matrix M (Alg. 2: pairwise center distances,
//           each row sorted by distance, own center first, ties by index).
//           Block 0 publishes the palette and the iteration record.
//   search  one block per CU.  Each lane takes one point, starts from its
//           previous center p, walks M[p] and stops at the first center
//           with d(c_p,c_t)^2 >= 4 d(x,c_p)^2 (sort-means).  The new
//           membership is written back and count*(R,G,B,1) is added into
//           per-block LDS accumulators, which are flushed once per block
//           with 64-bit device atomics (second level of the reduction).
//
// The full-search comparator fuses the update into its search kernel (one
// launch per iteration): every block recomputes the K centers from the
// totals itself, which is cheap, and a full search needs no M.
//
// State records and palettes are double-buffered by step parity and the
// totals are triple-buffered, so no launch reads what another block of the
// same launch writes.  After the last step a single-block kernel applies the
// final update and copies the result to the public slot 0.
#include "wsm_internal.h"

namespace wsm {

struct IterArgs {
    StateView sv;
    Points pts;
    int k;
    int grid;          // blocks of the search kernel (partials per step)
    double eps;
};

// ---------------------------------------------------------------------------
// Update phase, run by every block of a rows / fused / final launch.
// Produces the centers entering the search of step i in `cen` (LDS) and the
// record after the update.  Block `writer` publishes palette, record and the
// history entry.  Returns the record (same in every thread of every block).
template <int NT>
__device__ Record update_phase(const IterArgs &a, int i, float4 *cen, bool writer,
                               double *dscr, unsigned long long *uscr) {
    const int tid = threadIdx.x;
    const Header *hdr = a.sv.hdr;
    const Record rin = hdr->rec[i & 1];
    const float4 *pal_in = a.sv.pal + (size_t)(i & 1) * kMaxK;
    float4 *pal_out = a.sv.pal + (size_t)((i + 1) & 1) * kMaxK;
    Record r = rin;
    if (i == 0 || rin.converged) {
        for (int c = tid; c < a.k; c += NT) cen[c] = pal_in[c];
    } else {
        const unsigned long long *T = a.sv.totals + (size_t)((i - 1) % 3) * kMaxK * 4;
        for (int c = tid; c < a.k; c += NT) {
            const unsigned long long w = T[c * 4 + 3];
            if (w != 0ull) {
                const double dw = (double)w;
                cen[c] = make_float4((float)((double)T[c * 4 + 0] / dw),
                                     (float)((double)T[c * 4 + 1] / dw),
                                     (float)((double)T[c * 4 + 2] / dw), 0.0f);
            } else {
                cen[c] = pal_in[c];  // empty cluster keeps its center
            }
        }
        // Weighted SSE of step i-1 from the per-block partials, reduced by
        // the first wave in a fixed order (identical in every block).
        const double *sp = a.sv.sse_part + (size_t)((i - 1) & 1) * kMaxGrid;
        const unsigned long long *ep = a.sv.eval_part + (size_t)((i - 1) & 1) * kMaxGrid;
        if (tid < 64) {
            double s = 0.0;
            unsigned long long e = 0;
            for (int g = tid; g < a.grid; g += 64) {
                s += sp[g];
                e += ep[g];
            }
            for (int off = 32; off > 0; off >>= 1) {
                s += __shfl_xor(s, off, 64);
                e += __shfl_xor(e, off, 64);
            }
            if (tid == 0) {
                dscr[0] = s;
                uscr[0] = e;
            }
        }
        __syncthreads();
        const double sse = dscr[0] / (double)a.sv.hdr->n_pixels;
        const long long ev = (long long)uscr[0];
        const int t = rin.iters + 1;
        const bool stop = (sse == 0.0) || (t >= 2 && (rin.sse_last - sse) / sse <= a.eps);
        r.iters = t;
        r.converged = stop ? 1 : 0;
        r.sse_last = sse;
        if (writer && tid == 0 && t - 1 < kHistory) {
            a.sv.sse_hist[t - 1] = sse;
            a.sv.eval_hist[t - 1] = ev;
        }
    }
    __syncthreads();
    if (writer) {
        for (int c = tid; c < a.k; c += NT) pal_out[c] = cen[c];
        if (tid == 0) a.sv.hdr->rec[(i + 1) & 1] = r;
    }
    return r;
}

// ---------------------------------------------------------------------------
// Rows kernel: update + one row of M per block.  In map mode (map != 0) the
// centers are taken from the public palette and nothing but M is written.
__global__ __launch_bounds__(kRowThreads) void rows_kernel(IterArgs a, int i, int map) {
    __shared__ float4 cen[kMaxK];
    __shared__ unsigned long long key[kMaxK];
    __shared__ double dscr[4];
    __shared__ unsigned long long uscr[4];
    const int tid = threadIdx.x;
    const int row = blockIdx.x;
    if (map) {
        for (int c = tid; c < a.k; c += kRowThreads) cen[c] = a.sv.pal[c];
        __syncthreads();
    } else {
        const Record r = update_phase<kRowThreads>(a, i, cen, row == 0, dscr, uscr);
        if (r.converged) return;
        if (row == 0) {
            unsigned long long *T = a.sv.totals + (size_t)(i % 3) * kMaxK * 4;
            for (int c = tid; c < kMaxK * 4; c += kRowThreads) T[c] = 0ull;
        }
    }
    // Row `row` of M: centers ordered by (d(row, b), b != row, b).  The
    // float bits of a non-negative distance order like the value.
    const float4 ca = cen[row];
    for (int b = tid; b < a.k; b += kRowThreads) {
        const float4 cb = cen[b];
        const float d = sq_dist(ca.x, ca.y, ca.z, cb.x, cb.y, cb.z);
        key[b] = ((unsigned long long)__float_as_uint(d) << 32) |
                 ((unsigned long long)(b != row) << 8) | (unsigned long long)b;
    }
    __syncthreads();
    uint8_t *out = a.sv.rows + (size_t)row * kMaxK;
    for (int b = tid; b < a.k; b += kRowThreads) {
        const unsigned long long kb = key[b];
        int rank = 0;
        for (int c = 0; c < a.k; ++c) rank += key[c] < kb;
        out[rank] = (uint8_t)b;
    }
}

// ---------------------------------------------------------------------------
// Point access.
__device__ __forceinline__ void load_point(const Points &P, int64_t idx, float &x,
                                           float &y, float &z, uint32_t &cnt) {
    if (P.is_pixels) {
        const uint8_t *px = P.rgb + idx * 3;
        x = (float)px[0];
        y = (float)px[1];
        z = (float)px[2];
        cnt = 1u;
    } else {
        unpack_key(P.colors[idx], x, y, z);
        cnt = P.counts[idx];
    }
}

// Full search over all K centers with the same tie key.
__device__ __forceinline__ int full_scan(float x, float y, float z, int p, int K,
                                         const float4 *cen, float &best_d, uint32_t &ev) {
    const float4 cp = cen[p];
    float bd = sq_dist(x, y, z, cp.x, cp.y, cp.z);
    int best = p;
    for (int t = 0; t < K; ++t) {
        if (t == p) continue;
        const float4 ct = cen[t];
        const float d = sq_dist(x, y, z, ct.x, ct.y, ct.z);
        if (better_center(d, bd, t, best, p)) {
            bd = d;
            best = t;
        }
    }
    ev += (uint32_t)K;
    best_d = bd;
    return best;
}

// Search over this block's contiguous chunk of points, accumulation into
// LDS, flush of the block's totals and partials.
template <bool FULL>
__device__ void search_phase(const IterArgs &a, int i, const float4 *cen,
                             unsigned long long *acc, double *dscr,
                             unsigned long long *uscr) {
    const int tid = threadIdx.x;
    const int g = blockIdx.x;
    for (int c = tid; c < a.k * 4; c += kSearchThreads) acc[c] = 0ull;
    __syncthreads();
    const int64_t n = a.pts.n;
    int64_t chunk = (n + a.grid - 1) / a.grid;
    chunk = (chunk + 63) / 64 * 64;
    const int64_t start = (int64_t)g * chunk;
    const int64_t end = (start + chunk) < n ? (start + chunk) : n;
    double sse = 0.0;
    uint32_t ev = 0;
    for (int64_t idx = start + tid; idx < end; idx += kSearchThreads) {
        float x, y, z;
        uint32_t cnt;
        load_point(a.pts, idx, x, y, z, cnt);
        const int p = a.sv.m[idx];
        float bd;
        int best;
        if (FULL)
            best = full_scan(x, y, z, p, a.k, cen, bd, ev);
        else
            best = sm_scan(x, y, z, p, a.k, cen, a.sv.rows, bd, ev);
        a.sv.m[idx] = (uint8_t)best;
        sse += (double)cnt * (double)bd;
        const unsigned long long c64 = cnt;
        atomicAdd(&acc[best * 4 + 0], c64 * (unsigned long long)x);
        atomicAdd(&acc[best * 4 + 1], c64 * (unsigned long long)y);
        atomicAdd(&acc[best * 4 + 2], c64 * (unsigned long long)z);
        atomicAdd(&acc[best * 4 + 3], c64);
    }
    __syncthreads();
    unsigned long long *T = a.sv.totals + (size_t)(i % 3) * kMaxK * 4;
    for (int c = tid; c < a.k * 4; c += kSearchThreads) {
        const unsigned long long v = acc[c];
        if (v != 0ull) atomicAdd(&T[c], v);
    }
    const double s = block_sum_double<kSearchThreads>(sse, dscr);
    const unsigned long long e = block_sum_u64<kSearchThreads>((unsigned long long)ev, uscr);
    if (tid == 0) {
        a.sv.sse_part[(size_t)(i & 1) * kMaxGrid + g] = s;
        a.sv.eval_part[(size_t)(i & 1) * kMaxGrid + g] = e;
    }
}

// Sort-means search of step i (after rows_kernel of step i).
__global__ __launch_bounds__(kSearchThreads) void search_kernel(IterArgs a, int i) {
    __shared__ float4 cen[kMaxK];
    __shared__ unsigned long long acc[kMaxK * 4];
    __shared__ double dscr[kSearchThreads / 64];
    __shared__ unsigned long long uscr[kSearchThreads / 64];
    const int tid = threadIdx.x;
    const Record r = a.sv.hdr->rec[(i + 1) & 1];
    if (r.converged) return;
    const float4 *pal = a.sv.pal + (size_t)((i + 1) & 1) * kMaxK;
    for (int c = tid; c < a.k; c += kSearchThreads) cen[c] = pal[c];
    __syncthreads();
    search_phase<false>(a, i, cen, acc, dscr, uscr);
}

// Full-search comparator: update of step i-1 fused with the search of step i.
__global__ __launch_bounds__(kSearchThreads) void full_step_kernel(IterArgs a, int i) {
    __shared__ float4 cen[kMaxK];
    __shared__ unsigned long long acc[kMaxK * 4];
    __shared__ double dscr[kSearchThreads / 64];
    __shared__ unsigned long long uscr[kSearchThreads / 64];
    const int tid = threadIdx.x;
    const Record r = update_phase<kSearchThreads>(a, i, cen, blockIdx.x == 0, dscr, uscr);
    if (r.converged) return;
    if (blockIdx.x == 0) {
        unsigned long long *T = a.sv.totals + (size_t)((i + 1) % 3) * kMaxK * 4;
        for (int c = tid; c < kMaxK * 4; c += kSearchThreads) T[c] = 0ull;
    }
    search_phase<true>(a, i, cen, acc, dscr, uscr);
}

// Final update after the last step of a call (one block).  Publishes the
// palette and record to slot 0 and clears totals[0] for the next call.
__global__ __launch_bounds__(kRowThreads) void final_kernel(IterArgs a, int i) {
    __shared__ float4 cen[kMaxK];
    __shared__ double dscr[4];
    __shared__ unsigned long long uscr[4];
    const int tid = threadIdx.x;
    const Record r = update_phase<kRowThreads>(a, i, cen, true, dscr, uscr);
    __syncthreads();
    for (int c = tid; c < a.k; c += kRowThreads) a.sv.pal[c] = cen[c];
    unsigned long long *T0 = a.sv.totals;
    for (int c = tid; c < kMaxK * 4; c += kRowThreads) T0[c] = 0ull;
    if (tid == 0) {
        a.sv.hdr->rec[0] = r;
        a.sv.hdr->info[0] = r.iters;
        a.sv.hdr->info[1] = r.converged;
        a.sv.hdr->info[2] = r.err;
        a.sv.hdr->info[3] = 0;
    }
}

// State initialisation: header, palette slot 0, cleared records, totals,
// histories and memberships.
__global__ void init_state_kernel(StateView sv, int k, int points, int grid,
                                  int64_t n_points, int64_t n_pixels,
                                  const float *__restrict__ init_palette) {
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (gt == 0) {
        Header *h = sv.hdr;
        h->magic = kMagic;
        h->k = k;
        h->points = points;
        h->grid = grid;
        h->n_points = n_points;
        h->n_pixels = n_pixels;
        for (int j = 0; j < 4; ++j) h->reserved[j] = 0ull;
        Record z;
        z.iters = 0;
        z.converged = 0;
        z.err = 0;
        z.pad = 0;
        z.sse_last = 0.0;
        z.pad2 = 0.0;
        h->rec[0] = z;
        h->rec[1] = z;
        for (int j = 0; j < 4; ++j) h->info[j] = 0;
    }
    for (int64_t c = gt; c < 2 * kMaxK; c += stride) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (c < k) v = make_float4(init_palette[3 * c], init_palette[3 * c + 1],
                                   init_palette[3 * c + 2], 0.f);
        sv.pal[c] = v;
    }
    for (int64_t c = gt; c < 3 * kMaxK * 4; c += stride) sv.totals[c] = 0ull;
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

extern "C" int wsm_gather_palette(const uint32_t *colors, int64_t n_colors,
                                  const int32_t *indices, int k, float *palette,
                                  hipStream_t stream) {
    if (!colors || !indices || !palette || n_colors < 1 || k < 1 || k > kMaxK) return WSM_EINVAL;
    (void)hipGetLastError();
    gather_palette_kernel<<<dim3(1), dim3(kMaxK), 0, stream>>>(colors, n_colors, indices, k,
                                                               palette);
    return hipGetLastError() == hipSuccess ? WSM_OK : WSM_EHIP;
}

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
    int grid = cus;
    if (grid > kMaxGrid) grid = kMaxGrid;
    const int64_t need = (n_points + kSearchThreads - 1) / kSearchThreads;
    if (need < grid) grid = (int)need;
    if (grid < 1) grid = 1;
    StateView sv = make_view(state);
    (void)hipGetLastError();
    init_state_kernel<<<dim3(256), dim3(256), 0, stream>>>(sv, k, points, grid, n_points,
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
    prob->grid = grid;
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

extern "C" int wsm_iterate(const wsm_problem *prob, int max_iters, double eps,
                           hipStream_t stream) {
    int rc = check_iter_args(prob, max_iters, eps);
    if (rc != WSM_OK) return rc;
    const IterArgs a = make_args(prob, eps);
    (void)hipGetLastError();
    for (int i = 0; i < max_iters; ++i) {
        timing_before(WSM_KERNEL_ROWS, stream);
        rows_kernel<<<dim3(a.k), dim3(kRowThreads), 0, stream>>>(a, i, 0);
        timing_after(WSM_KERNEL_ROWS, stream);
        timing_before(WSM_KERNEL_SEARCH, stream);
        search_kernel<<<dim3(a.grid), dim3(kSearchThreads), 0, stream>>>(a, i);
        timing_after(WSM_KERNEL_SEARCH, stream);
    }
    final_kernel<<<dim3(1), dim3(kRowThreads), 0, stream>>>(a, max_iters);
    if (hipGetLastError() != hipSuccess) return WSM_EHIP;
    return WSM_OK;
}

extern "C" int wsm_iterate_full(const wsm_problem *prob, int max_iters, double eps,
                                hipStream_t stream) {
    int rc = check_iter_args(prob, max_iters, eps);
    if (rc != WSM_OK) return rc;
    const IterArgs a = make_args(prob, eps);
    (void)hipGetLastError();
    for (int i = 0; i < max_iters; ++i) {
        timing_before(WSM_KERNEL_FULL_STEP, stream);
        full_step_kernel<<<dim3(a.grid), dim3(kSearchThreads), 0, stream>>>(a, i);
        timing_after(WSM_KERNEL_FULL_STEP, stream);
    }
    final_kernel<<<dim3(1), dim3(kRowThreads), 0, stream>>>(a, max_iters);
    if (hipGetLastError() != hipSuccess) return WSM_EHIP;
    return WSM_OK;
}

extern "C" int wsm_state_views(const wsm_problem *prob, wsm_views *views) {
    if (!views) return WSM_EINVAL;
    int rc = check_problem(prob);
    if (rc != WSM_OK) return rc;
    const StateView sv = make_view(prob->state);
    views->palette = (const float *)sv.pal;
    views->membership = sv.m;
    views->sse_history = sv.sse_hist;
    views->evals_history = (const int64_t *)sv.eval_hist;
    views->info = sv.hdr->info;
    return WSM_OK;
}

// Launch helper used by the pixel map: M for the public palette.
int wsm_internal_rows_for_map(const wsm_problem *prob, hipStream_t stream) {
    const IterArgs a = make_args(prob, 0.0);
    rows_kernel<<<dim3(a.k), dim3(kRowThreads), 0, stream>>>(a, 0, 1);
    return hipGetLastError() == hipSuccess ? WSM_OK : WSM_EHIP;
}
