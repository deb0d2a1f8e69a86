// Differentiable form of the quantizer's distortion on gfx950: the weighted
// SSE of Eq. 1 taken over the pixels themselves,
//     D = (1/N) sum_p ||x_p - c_{m(p)}||^2,
// for a batch of images with float32 pixel colors x, palettes c and frozen
// assignments m (the pixel map), and its adjoint
//     dD/dx_p = (2/N) (x_p - c_{m(p)}),   dD/dc_k = (2/N) sum_{m(p)=k} (c_k - x_p).
// D is piecewise quadratic in (x, c); away from assignment ties these are
// its derivatives.
//
// Both passes are HBM-bound streams over the pixels (12 B of color and 1 B
// of index in; 12 B of gradient out for the adjoint).  Each block takes a
// tile of kAdjTile pixels of one image and keeps its image's palette in
// LDS; differences and sums are in float64 (the difference of two float32
// values is exact in float64).  Per-block partials go to the workspace and
// are summed in a fixed order by a second launch, so D is reproducible; the
// palette gradient's per-block sums use LDS float64 atomics, one per run of
// equal centers within a wave (a segmented wave sum first).
#include "sm_block.h"

namespace wsm {

constexpr int kAdjThreads = 256;
constexpr int kAdjPpt = 16;                         // pixels per thread
constexpr int kAdjTile = kAdjThreads * kAdjPpt;     // pixels per block

struct AdjLayout {
    int64_t tiles;          // blocks per image
    size_t off_d, off_c, bytes;
};

static AdjLayout adj_layout(int batch, int64_t n, int k) {
    AdjLayout L;
    L.tiles = (n + kAdjTile - 1) / kAdjTile;
    L.off_d = 0;
    L.off_c = align_up((size_t)batch * L.tiles * 8, 256);
    L.bytes = align_up(L.off_c + (size_t)batch * L.tiles * k * 3 * 8, 256);
    return L;
}

// Segmented inclusive sums of three float64 values over the wave (as
// wave_seg_sum2 for two 64-bit integers): a segment starts at lanes with
// head != 0, and the last lane of each segment ends with the segment's sums.
template <int CTRL>
__device__ __forceinline__ void seg_step_sum3_f64(int lane, int &f, double &a, double &b,
                                                  double &c) {
    const int tf = dpp_i32<CTRL>(f);
    const double ta = dpp_f64<CTRL>(a);
    const double tb = dpp_f64<CTRL>(b);
    const double tc = dpp_f64<CTRL>(c);
    if (dpp_takes<CTRL>(lane)) {
        if (!f) {
            a += ta;
            b += tb;
            c += tc;
        }
        f |= tf;
    }
}

__device__ __forceinline__ void wave_seg_sum3_f64(int head, double &a, double &b, double &c) {
    const int lane = threadIdx.x & 63;
    int f = head;
    seg_step_sum3_f64<kDppRowShr1>(lane, f, a, b, c);
    seg_step_sum3_f64<kDppRowShr2>(lane, f, a, b, c);
    seg_step_sum3_f64<kDppRowShr4>(lane, f, a, b, c);
    seg_step_sum3_f64<kDppRowShr8>(lane, f, a, b, c);
    seg_step_sum3_f64<kDppRowBcast15>(lane, f, a, b, c);
    seg_step_sum3_f64<kDppRowBcast31>(lane, f, a, b, c);
}

__device__ __forceinline__ void load_palette(const float *__restrict__ pal, int k, float4 *cp) {
    for (int c = threadIdx.x; c < kMaxK; c += kAdjThreads)
        cp[c] = c < k ? make_float4(pal[3 * c], pal[3 * c + 1], pal[3 * c + 2], 0.f)
                      : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Block b of image i: sum over its pixels of ||x_p - c_m(p)||^2 (float64),
// reduced in a fixed order (lanes, then waves), into part[i][b].
// Four consecutive pixels from a lane's 16-byte-aligned base q: their 12
// float32 colors (three 16-byte loads) and their 4 palette indices (one
// 4-byte load).  VEC launches need n % 4 == 0 and 16-byte aligned x.
__device__ __forceinline__ void load_quad(const float *xi, const uint8_t *mi, int64_t q,
                                          float (&xv)[12], uint32_t &m4) {
    const float4 *src = (const float4 *)(xi + 3 * q);
    const float4 a = src[0], b = src[1], c = src[2];
    const float v[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
#pragma unroll
    for (int e = 0; e < 12; ++e) xv[e] = v[e];
    m4 = *(const uint32_t *)(mi + q);
}

template <bool VEC>
__global__ __launch_bounds__(kAdjThreads) void distortion_partial_kernel(
    const float *__restrict__ x, const uint8_t *__restrict__ idx, const float *__restrict__ pal,
    int64_t n, int k, int64_t tiles, double *__restrict__ part) {
    __shared__ float4 cp[kMaxK];
    __shared__ double scr[kAdjThreads / 64];
    const int64_t img = blockIdx.y;
    load_palette(pal + img * k * 3, k, cp);
    __syncthreads();
    const float *xi = x + img * n * 3;
    const uint8_t *mi = idx + img * n;
    const int64_t p0 = (int64_t)blockIdx.x * kAdjTile;
    double s = 0.0;
    if (VEC) {
#pragma unroll 2
        for (int it = 0; it < kAdjPpt / 4; ++it) {
            const int64_t q = p0 + ((int64_t)it * kAdjThreads + threadIdx.x) * 4;
            if (q < n) {  // n % 4 == 0: all four pixels are in the image
                float xv[12];
                uint32_t m4;
                load_quad(xi, mi, q, xv, m4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float4 c = cp[(m4 >> (8 * e)) & 0xFFu];
                    const double dx = (double)xv[3 * e] - (double)c.x;
                    const double dy = (double)xv[3 * e + 1] - (double)c.y;
                    const double dz = (double)xv[3 * e + 2] - (double)c.z;
                    s += dx * dx + dy * dy + dz * dz;
                }
            }
        }
    } else {
#pragma unroll 4
        for (int j = 0; j < kAdjPpt; ++j) {
            const int64_t p = p0 + j * kAdjThreads + threadIdx.x;
            if (p < n) {
                const float4 c = cp[mi[p]];
                const double dx = (double)xi[3 * p] - (double)c.x;
                const double dy = (double)xi[3 * p + 1] - (double)c.y;
                const double dz = (double)xi[3 * p + 2] - (double)c.z;
                s += dx * dx + dy * dy + dz * dz;
            }
        }
    }
    const double t = block_sum_f64<kAdjThreads>(s, scr);
    if (threadIdx.x == 0) part[img * tiles + blockIdx.x] = t;
}

// D of image i: its block partials summed in order, divided by n.
__global__ __launch_bounds__(64) void distortion_reduce_kernel(const double *__restrict__ part,
                                                               int64_t tiles, int64_t n,
                                                               double *__restrict__ d_out) {
    const int64_t img = blockIdx.x;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < tiles; b += 64) s += part[img * tiles + b];
    s = wave_sum_f64(s);
    if (threadIdx.x == 63) d_out[img] = s / (double)n;
}

// Adjoint, block b of image i: dD/dx for its pixels (when grad_x is not
// null) and the sums over its pixels of x_p - c_m(p) per center, into
// part[i][b][k][3] (when the palette gradient is wanted).
template <bool VEC>
__global__ __launch_bounds__(kAdjThreads) void distortion_grad_kernel(
    const float *__restrict__ x, const uint8_t *__restrict__ idx, const float *__restrict__ pal,
    int64_t n, int k, int64_t tiles, const double *__restrict__ grad_d, float *__restrict__ grad_x,
    double *__restrict__ part) {
    __shared__ float4 cp[kMaxK];
    __shared__ double acc[kMaxK * 3];
    const int64_t img = blockIdx.y;
    load_palette(pal + img * k * 3, k, cp);
    if (part)
        for (int c = threadIdx.x; c < k * 3; c += kAdjThreads) acc[c] = 0.0;
    __syncthreads();
    const double scale = 2.0 * grad_d[img] / (double)n;
    const float *xi = x + img * n * 3;
    const uint8_t *mi = idx + img * n;
    float *gxi = grad_x ? grad_x + img * n * 3 : nullptr;
    const int64_t p0 = (int64_t)blockIdx.x * kAdjTile;
    if (VEC) {
        for (int it = 0; it < kAdjPpt / 4; ++it) {
            const int64_t q = p0 + ((int64_t)it * kAdjThreads + threadIdx.x) * 4;
            const bool valid = q < n;  // n % 4 == 0: all four pixels or none
            float xv[12] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            uint32_t m4 = 0u;
            if (valid) load_quad(xi, mi, q, xv, m4);
            double d[12];
            int m[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                m[e] = valid ? (int)((m4 >> (8 * e)) & 0xFFu) : -1;
                const float4 c = valid ? cp[m[e]] : make_float4(0.f, 0.f, 0.f, 0.f);
                d[3 * e] = valid ? (double)xv[3 * e] - (double)c.x : 0.0;
                d[3 * e + 1] = valid ? (double)xv[3 * e + 1] - (double)c.y : 0.0;
                d[3 * e + 2] = valid ? (double)xv[3 * e + 2] - (double)c.z : 0.0;
            }
            if (gxi && valid) {
                float g[12];
#pragma unroll
                for (int e = 0; e < 12; ++e) g[e] = (float)(scale * d[e]);
                float4 *dst = (float4 *)(gxi + 3 * q);
                dst[0] = make_float4(g[0], g[1], g[2], g[3]);
                dst[1] = make_float4(g[4], g[5], g[6], g[7]);
                dst[2] = make_float4(g[8], g[9], g[10], g[11]);
            }
            if (part) {  // uniform: every lane of the wave takes part
                // pixel e of every lane in turn: neighbouring lanes' pixels
                // are 4 apart and mostly share a center as well
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    wave_seg_sum3_f64(run_head(m[e]), d[3 * e], d[3 * e + 1], d[3 * e + 2]);
                    if (run_tail(m[e], valid)) {
                        atomicAdd(&acc[3 * m[e]], d[3 * e]);
                        atomicAdd(&acc[3 * m[e] + 1], d[3 * e + 1]);
                        atomicAdd(&acc[3 * m[e] + 2], d[3 * e + 2]);
                    }
                }
            }
        }
    } else {
#pragma unroll 4
    for (int j = 0; j < kAdjPpt; ++j) {
        const int64_t p = p0 + j * kAdjThreads + threadIdx.x;
        const bool valid = p < n;
        int m = -1;
        double dx = 0.0, dy = 0.0, dz = 0.0;
        if (valid) {
            m = mi[p];
            const float4 c = cp[m];
            dx = (double)xi[3 * p] - (double)c.x;
            dy = (double)xi[3 * p + 1] - (double)c.y;
            dz = (double)xi[3 * p + 2] - (double)c.z;
            if (gxi) {
                gxi[3 * p] = (float)(scale * dx);
                gxi[3 * p + 1] = (float)(scale * dy);
                gxi[3 * p + 2] = (float)(scale * dz);
            }
        }
        if (part) {  // uniform: every lane of the wave takes part
            // Neighbouring pixels mostly share a center: the wave sums each
            // run of equal centers first, and the run's last lane adds it.
            wave_seg_sum3_f64(run_head(m), dx, dy, dz);
            if (run_tail(m, valid)) {
                atomicAdd(&acc[3 * m], dx);
                atomicAdd(&acc[3 * m + 1], dy);
                atomicAdd(&acc[3 * m + 2], dz);
            }
        }
    }
    }
    if (part) {
        __syncthreads();
        double *dst = part + (img * tiles + blockIdx.x) * k * 3;
        for (int c = threadIdx.x; c < k * 3; c += kAdjThreads) dst[c] = acc[c];
    }
}

// dD/dc of image i: for each (center, channel) e, the block sums added in a
// fixed order -- wave w of kRedWaves sums blocks w, w + kRedWaves, ... in
// order (lane l: element e0 + l), then the waves' sums are added in wave
// order -- times -2 g / n.  The loads of kRedBatch blocks are issued
// together.
constexpr int kRedWaves = kAdjThreads / 64;
constexpr int kRedBatch = 8;

__global__ __launch_bounds__(kAdjThreads) void grad_palette_reduce_kernel(
    const double *__restrict__ part, int64_t tiles, int64_t n, int k,
    const double *__restrict__ grad_d, float *__restrict__ grad_pal) {
    __shared__ double ws[kRedWaves][64];
    const int64_t img = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;  // center * 3 + channel
    const bool in = e < k * 3;
    const double *pi = part + img * tiles * k * 3 + e;
    double s = 0.0;
    for (int64_t b0 = wave; b0 < tiles; b0 += (int64_t)kRedWaves * kRedBatch) {
        double v[kRedBatch];
#pragma unroll
        for (int u = 0; u < kRedBatch; ++u) {
            const int64_t b = b0 + (int64_t)u * kRedWaves;
            v[u] = in && b < tiles ? pi[b * k * 3] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kRedBatch; ++u) s += v[u];
    }
    ws[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && in) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kRedWaves; ++w) t += ws[w][lane];
        grad_pal[img * k * 3 + e] = (float)(-2.0 * grad_d[img] / (double)n * t);
    }
}

}  // namespace wsm

using namespace wsm;

static int adj_check(const float *x, const uint8_t *index, const float *palette, int batch,
                     int64_t n_pixels, int k, void *workspace, size_t workspace_bytes) {
    if (!x || !index || !palette || !workspace) return WSM_EINVAL;
    if (batch < 1 || batch > 65535 || n_pixels < 1 || k < 1 || k > kMaxK) return WSM_EINVAL;
    if (n_pixels > (int64_t)0xFFFFFFFFll) return WSM_EINVAL;
    if (((uintptr_t)x & 3u) != 0u || ((uintptr_t)palette & 3u) != 0u) return WSM_EINVAL;
    if (((uintptr_t)workspace & 15u) != 0u) return WSM_EINVAL;
    if (workspace_bytes < adj_layout(batch, n_pixels, k).bytes) return WSM_ENOSPC;
    return WSM_OK;
}

// Whether the kernels take four pixels per lane with 16-byte accesses:
// every image's colors (and gradients) 16-byte aligned and its indices
// 4-byte aligned.
static bool adj_vec(const float *x, const uint8_t *index, const float *grad_x, int64_t n) {
    return n % 4 == 0 && ((uintptr_t)x & 15u) == 0u && ((uintptr_t)index & 3u) == 0u &&
           (!grad_x || ((uintptr_t)grad_x & 15u) == 0u);
}

extern "C" int wsm_distortion_workspace_bytes(int batch, int64_t n_pixels, int k, size_t *bytes) {
    if (!bytes || batch < 1 || batch > 65535 || n_pixels < 1 || n_pixels > (int64_t)0xFFFFFFFFll ||
        k < 1 || k > kMaxK)
        return WSM_EINVAL;
    *bytes = adj_layout(batch, n_pixels, k).bytes;
    return WSM_OK;
}

extern "C" int wsm_distortion(const float *x, const uint8_t *index, const float *palette,
                              int batch, int64_t n_pixels, int k, double *d_out, void *workspace,
                              size_t workspace_bytes, hipStream_t stream) {
    int rc = adj_check(x, index, palette, batch, n_pixels, k, workspace, workspace_bytes);
    if (rc != WSM_OK) return rc;
    if (!d_out || ((uintptr_t)d_out & 7u) != 0u) return WSM_EINVAL;
    const AdjLayout L = adj_layout(batch, n_pixels, k);
    double *part = (double *)((char *)workspace + L.off_d);
    (void)hipGetLastError();
    if (adj_vec(x, index, nullptr, n_pixels))
        distortion_partial_kernel<true><<<dim3((unsigned)L.tiles, (unsigned)batch),
                                          dim3(kAdjThreads), 0, stream>>>(x, index, palette,
                                                                          n_pixels, k, L.tiles,
                                                                          part);
    else
        distortion_partial_kernel<false><<<dim3((unsigned)L.tiles, (unsigned)batch),
                                           dim3(kAdjThreads), 0, stream>>>(x, index, palette,
                                                                           n_pixels, k, L.tiles,
                                                                           part);
    distortion_reduce_kernel<<<dim3((unsigned)batch), dim3(64), 0, stream>>>(part, L.tiles,
                                                                            n_pixels, d_out);
    return hipGetLastError() == hipSuccess ? WSM_OK : WSM_EHIP;
}

extern "C" int wsm_distortion_backward(const float *x, const uint8_t *index, const float *palette,
                                       int batch, int64_t n_pixels, int k, const double *grad_d,
                                       float *grad_x, float *grad_palette, void *workspace,
                                       size_t workspace_bytes, hipStream_t stream) {
    int rc = adj_check(x, index, palette, batch, n_pixels, k, workspace, workspace_bytes);
    if (rc != WSM_OK) return rc;
    if (!grad_d || ((uintptr_t)grad_d & 7u) != 0u) return WSM_EINVAL;
    if (!grad_x && !grad_palette) return WSM_EINVAL;
    if ((grad_x && ((uintptr_t)grad_x & 3u) != 0u) ||
        (grad_palette && ((uintptr_t)grad_palette & 3u) != 0u))
        return WSM_EINVAL;
    const AdjLayout L = adj_layout(batch, n_pixels, k);
    double *part = grad_palette ? (double *)((char *)workspace + L.off_c) : nullptr;
    (void)hipGetLastError();
    if (adj_vec(x, index, grad_x, n_pixels))
        distortion_grad_kernel<true><<<dim3((unsigned)L.tiles, (unsigned)batch),
                                       dim3(kAdjThreads), 0, stream>>>(
            x, index, palette, n_pixels, k, L.tiles, grad_d, grad_x, part);
    else
        distortion_grad_kernel<false><<<dim3((unsigned)L.tiles, (unsigned)batch),
                                        dim3(kAdjThreads), 0, stream>>>(
            x, index, palette, n_pixels, k, L.tiles, grad_d, grad_x, part);
    if (grad_palette)
        grad_palette_reduce_kernel<<<dim3((unsigned)((k * 3 + 63) / 64), (unsigned)batch),
                                     dim3(kAdjThreads), 0, stream>>>(part, L.tiles, n_pixels, k,
                                                                     grad_d, grad_palette);
    return hipGetLastError() == hipSuccess ? WSM_OK : WSM_EHIP;
}
