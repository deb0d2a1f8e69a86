// Pixel mapping (Sec. 1: the second phase of color quantization) and the MSE
// of Sec. 3.1, on gfx950.
//
//   rows    the neighbour matrix M of the final palette, one row per block.
//   assign  a sort-means scan of every unique color against the final palette,
//           starting from the color's last membership, as in the iteration
//           search for large K (sm_block.h): the row heads of M and their
//           distances in LDS, a wave's scans over them spread over its lanes,
//           the rare longer ones finished by whole waves.  One block per CU.
//           Each choice is made final in float64 against the float64
//           palette (decide64), and the palette index is scattered into a
//           2^24-entry byte table laid out in 4 x 4 x 4 color cells
//           (lut_index); count * float64 distance is summed per block for
//           the MSE.
//   gather  16 pixels per lane: three 16-byte loads, 16 table lookups, one
//           16-byte store of indices (and 48 bytes of rounded palette colors
//           when asked for).  Block 0 also sums the MSE partials.
#include "sm_block.h"

int wsm_internal_check_problem(const wsm_problem *prob);
int wsm_internal_palette_rows(void *state, int k, hipStream_t stream);

namespace wsm {

constexpr int kMapThreads = 256;

// Position of color (r, g, b) in the lookup table: the table is laid out in
// 4 x 4 x 4 color cells of 64 bytes each, so that similar colors share cache
// lines and the part of the table an image touches stays small.
__device__ __forceinline__ uint32_t lut_index(uint32_t r, uint32_t g, uint32_t b) {
    const uint32_t cell = ((r >> 2) << 12) | ((g >> 2) << 6) | (b >> 2);
    return (cell << 6) | ((r & 3u) << 4) | ((g & 3u) << 2) | (b & 3u);
}

__device__ __forceinline__ uint32_t lut_index_key(uint32_t key) {
    return lut_index((key >> 16) & 0xFFu, (key >> 8) & 0xFFu, key & 0xFFu);
}
constexpr int kGatherPpt = 16;

// FLAT (K >= kDeferMinK, as in the iteration search): flattened scans over
// the row heads, long scans deferred.  Otherwise each lane scans its color's
// whole row in LDS (sm_scan).
template <bool FLAT>
__global__ __launch_bounds__(kSearchThreads) void map_assign_kernel(
    StateView sv, const uint32_t *__restrict__ colors, const uint32_t *__restrict__ counts,
    int64_t n, int K, uint8_t *__restrict__ lut) {
    constexpr int NT = kSearchThreads;
    constexpr int NW = NT / 64;
    __shared__ float4 cen[kMaxK];
    __shared__ double4 cen64[kMaxK];
    // rows of M: their heads (FLAT) or whole
    __shared__ __align__(16) uint8_t Ms[kMaxK * (FLAT ? kRowPrefix : kRowStride)];
    __shared__ __align__(16) float Dd[FLAT ? kMaxK * kRowDist : 4];  // the heads' distances
    __shared__ FlatScratch fs[FLAT ? NW : 1];
    __shared__ DeferQueue dq;
    __shared__ double dscr[NW];
    __shared__ uint32_t next;  // the block's next slot
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    // the 64-color chunks b, b + grid, b + 2 grid, ... (every block samples
    // the whole key range, so the blocks get similar work), its slots
    const int64_t grid = gridDim.x;
    const int64_t chunks = (n + 63) / 64;
    const int64_t ns = chunks > (int64_t)blockIdx.x ? (chunks - blockIdx.x + grid - 1) / grid : 0;
    int flags = 0;
    for (int c = tid; c < K; c += NT) {
        const double4 c64 = sv.pal64[c];
        cen[c] = sv.pal[c];
        cen64[c] = c64;
        flags |= center_flags(c64);
    }
    RowRegs<NT> R;
    fetch_rows<NT, FLAT>(sv.rows, K, R);
    store_rows<NT, FLAT>(R, K, Ms);
    if (FLAT)
        for (int q = tid; q < K * (kRowDist / 4); q += NT)
            ((uint4 *)Dd)[q] = ((const uint4 *)sv.rowd)[q];
    if (tid == 0) {
        dq.n = 0u;
        next = 0u;
    }
    const int mode = block_mode(flags);
    double acc = 0.0;
    uint32_t ev = 0;
    // Each wave takes the block's slots one at a time from an LDS counter,
    // the next slot's colors loaded a round ahead, so that waves whose
    // colors scan long take fewer slots.
    int64_t dslot = 0;
    uint32_t kd = 0u, cd = 0u;
    int pd = 0;
    auto take = [&]() {
        uint32_t t = 0u;
        if (lane == 0) t = atomicAdd(&next, 1u);
        dslot = (int64_t)__builtin_amdgcn_readfirstlane(t);
        const int64_t idx = ((int64_t)blockIdx.x + dslot * grid) * 64 + lane;
        kd = 0u;
        cd = 0u;
        pd = 0;
        if (dslot < ns && idx < n) {
            kd = colors[idx];
            cd = counts[idx];
            pd = sv.m[idx];
        }
    };
    take();
#pragma unroll 1
    for (;;) {
        const uint32_t kr = kd, cr = cd;
        const int pr = pd;
        const int64_t slot = dslot;
        if (slot >= ns) break;  // wave-uniform
        take();
        {
            const int64_t idx = ((int64_t)blockIdx.x + slot * grid) * 64 + lane;
            const bool valid = idx < n;
            // the wave's scans over the row heads together; one that goes
            // past the head is deferred (or, with the queue full, carried on
            // by its lane)
            float thr = 0.f, bd = 0.f, s2 = kNoSkip, prev = 0.f, dj = kNoSkip;
            int best = 0;
            bool more = false;
            if (FLAT) {
                sm_scan_flat(valid, kr, pr, K, cen, Ms, Dd, fs[wave], thr, prev, bd, s2, dj,
                             best, ev, more);
            } else if (valid) {
                float x, y, z;
                unpack_key(kr, x, y, z);
                best = sm_scan(x, y, z, pr, K, cen, Ms, lds_row_stride(K), bd, prev, s2, dj,
                               ev);
            }
            bool done = true;
            if (FLAT && more) {
                const uint32_t q = atomicAdd(&dq.n, 1u);
                if (q < (uint32_t)kDeferCap) {
                    dq.idx[q] = (uint32_t)idx;
                    dq.key[q] = kr;
                    dq.cnt[q] = cr;
                    dq.bd[q] = __float_as_uint(bd);
                    dq.s2[q] = __float_as_uint(s2);
                    dq.pjb[q] = ((uint32_t)kRowPrefix << 16) | ((uint32_t)pr << 8) |
                                (uint32_t)best;
                    done = false;
                } else {
                    float x, y, z;
                    unpack_key(kr, x, y, z);
                    const RowView rv{Ms + pr * kRowPrefix, sv.rows + (size_t)pr * kRowStride,
                                     kRowPrefix};
                    int j = kRowPrefix;
                    dj = kNoSkip;
                    sm_scan_range(x, y, z, pr, K, cen, rv, thr, j, K, bd, best, s2, dj, ev);
                }
            }
            const bool fin = valid && done;
            const double d64 = decide64(fin, kr, pr, K, mode, cen64, best, bd, s2, prev, dj);
            if (fin) {
                lut[lut_index_key(kr)] = (uint8_t)best;
                acc += (double)cr * d64;
            }
        }
    }
    if (FLAT) {
        __syncthreads();
        finish_deferred<NT>(K, mode, cen, cen64, Ms, sv.rows, &dq, ev,
                            [&](uint32_t, uint32_t k, uint32_t c, int best, double d64) {
            lut[lut_index_key(k)] = (uint8_t)best;
            acc += (double)c * d64;
        });
    }
    const double s = block_sum_f64<NT>(acc, dscr);
    if (tid == 0) sv.map_part[blockIdx.x] = s;
}

template <bool VEC>
__global__ __launch_bounds__(kMapThreads) void map_gather_kernel(
    const uint8_t *__restrict__ rgb, int64_t n, const uint8_t *__restrict__ lut,
    uint8_t *__restrict__ index_out, uint8_t *__restrict__ rgb_out, double *__restrict__ mse_out,
    const double *__restrict__ map_part, int nparts, const double4 *__restrict__ pal, int K) {
    __shared__ uint32_t rpal[kMaxK];  // rounded palette colors, packed 0x00RRGGBB
    const int tid = threadIdx.x;
    if (rgb_out) {
        for (int c = tid; c < kMaxK; c += kMapThreads) {
            uint32_t v = 0u;
            if (c < K) {
                // the float64 palette rounded half to even, clamped to 0..255
                const double4 q = pal[c];
                const double r = fmin(fmax(rint(q.x), 0.0), 255.0);
                const double g = fmin(fmax(rint(q.y), 0.0), 255.0);
                const double b = fmin(fmax(rint(q.z), 0.0), 255.0);
                v = ((uint32_t)r << 16) | ((uint32_t)g << 8) | (uint32_t)b;
            }
            rpal[c] = v;
        }
        __syncthreads();
    }
    if (blockIdx.x == 0 && mse_out && tid < 64) {
        double s = 0.0;
        for (int g = tid; g < nparts; g += 64) s += map_part[g];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (tid == 0) *mse_out = s / (double)n;
    }
    const int64_t first = ((int64_t)blockIdx.x * kMapThreads + tid) * kGatherPpt;
    if (first >= n) return;
    if (VEC && first + kGatherPpt <= n) {
        const uint4 *src = (const uint4 *)(rgb + first * 3);
        const uint4 q0 = src[0], q1 = src[1], q2 = src[2];
        const uint32_t w[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y,
                                q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
        uint32_t idx4[4] = {0u, 0u, 0u, 0u};
        uint32_t out[12] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < kGatherPpt; ++j) {
            const int byte = 3 * j;
            const uint32_t r = (w[byte >> 2] >> (8 * (byte & 3))) & 0xFFu;
            const uint32_t g = (w[(byte + 1) >> 2] >> (8 * ((byte + 1) & 3))) & 0xFFu;
            const uint32_t b = (w[(byte + 2) >> 2] >> (8 * ((byte + 2) & 3))) & 0xFFu;
            const uint32_t id = lut[lut_index(r, g, b)];
            idx4[j >> 2] |= id << (8 * (j & 3));
            if (rgb_out) {
                const uint32_t c = rpal[id];
                const uint32_t ch[3] = {(c >> 16) & 0xFFu, (c >> 8) & 0xFFu, c & 0xFFu};
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const int ob = byte + e;
                    out[ob >> 2] |= ch[e] << (8 * (ob & 3));
                }
            }
        }
        *(uint4 *)(index_out + first) = make_uint4(idx4[0], idx4[1], idx4[2], idx4[3]);
        if (rgb_out) {
            uint4 *dst = (uint4 *)(rgb_out + first * 3);
            dst[0] = make_uint4(out[0], out[1], out[2], out[3]);
            dst[1] = make_uint4(out[4], out[5], out[6], out[7]);
            dst[2] = make_uint4(out[8], out[9], out[10], out[11]);
        }
    } else {
        for (int j = 0; j < kGatherPpt; ++j) {
            const int64_t q = first + j;
            if (q >= n) break;
            const uint8_t *px = rgb + q * 3;
            const uint32_t id = lut[lut_index(px[0], px[1], px[2])];
            index_out[q] = (uint8_t)id;
            if (rgb_out) {
                const uint32_t c = rpal[id];
                rgb_out[q * 3 + 0] = (uint8_t)((c >> 16) & 0xFFu);
                rgb_out[q * 3 + 1] = (uint8_t)((c >> 8) & 0xFFu);
                rgb_out[q * 3 + 2] = (uint8_t)(c & 0xFFu);
            }
        }
    }
}

}  // namespace wsm

using namespace wsm;

extern "C" int wsm_map_pixels(const wsm_problem *prob, const uint8_t *rgb, int64_t n_pixels,
                              uint8_t *lut, uint8_t *index_out, uint8_t *rgb_out,
                              double *mse_out, hipStream_t stream) {
    const int rc = wsm_internal_check_problem(prob);
    if (rc != WSM_OK) return rc;
    if (prob->points != WSM_POINTS_COLORS) return WSM_EINVAL;
    if (!rgb || !lut || !index_out) return WSM_EINVAL;
    if (n_pixels < 1 || n_pixels != prob->n_pixels) return WSM_EINVAL;
    StateView sv = make_view(prob->state);
    (void)hipGetLastError();
    // the state's search grid (one block per CU, fewer for small tables)
    int64_t nb = prob->grid;
    if (nb < 1) nb = 1;
    if (nb > kMaxGrid) nb = kMaxGrid;
    if (wsm_internal_palette_rows(prob->state, prob->k, stream) != WSM_OK) return WSM_EHIP;
    const auto assign = prob->k >= kDeferMinK ? map_assign_kernel<true> : map_assign_kernel<false>;
    WSM_LAUNCH(WSM_KERNEL_MAP_ASSIGN, assign, dim3((unsigned)nb), dim3(kSearchThreads), stream, sv,
               prob->colors, prob->counts, prob->n_points, prob->k, lut);
    if (hipGetLastError() != hipSuccess) return WSM_EHIP;
    const int64_t per_block = (int64_t)kMapThreads * kGatherPpt;
    const int64_t gb = (n_pixels + per_block - 1) / per_block;
    const bool vec = (((uintptr_t)rgb & 15u) == 0u) && (((uintptr_t)index_out & 15u) == 0u) &&
                     (!rgb_out || (((uintptr_t)rgb_out & 15u) == 0u));
    if (vec)
        WSM_LAUNCH(WSM_KERNEL_MAP_GATHER, map_gather_kernel<true>, dim3((unsigned)gb),
                   dim3(kMapThreads), stream, rgb, n_pixels, (const uint8_t *)lut, index_out,
                   rgb_out, mse_out, (const double *)sv.map_part, (int)nb, (const double4 *)sv.pal64,
                   prob->k);
    else
        WSM_LAUNCH(WSM_KERNEL_MAP_GATHER, map_gather_kernel<false>, dim3((unsigned)gb),
                   dim3(kMapThreads), stream, rgb, n_pixels, (const uint8_t *)lut, index_out,
                   rgb_out, mse_out, (const double *)sv.map_part, (int)nb, (const double4 *)sv.pal64,
                   prob->k);
    if (hipGetLastError() != hipSuccess) return WSM_EHIP;
    return WSM_OK;
}
