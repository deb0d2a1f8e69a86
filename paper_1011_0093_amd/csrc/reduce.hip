// Data reduction of the WSM quantizer (Sec. 2, "data sampling" and "sample
// weighting"): the unique 24-bit colors of an image with their pixel counts,
// emitted in ascending key order.
//
// Two kernels, both staging their hot data in LDS:
//   partition  one block per tile of T pixels.  Each pixel's key
//              R<<16 | G<<8 | B is split into a slice (top 9 bits, 512
//              slices) and a 15-bit low key.  An LDS histogram of the tile's
//              slices gives every pixel a rank; the low keys are written out
//              grouped by slice (a tile-local counting sort), 2 bytes per
//              pixel, together with a (offset, count) word per (slice, tile).
//   compact    one block per slice.  A 2^15-bin LDS histogram counts the
//              slice's low keys from every tile; the non-empty bins are
//              compacted in ascending order, and the slice's place in the
//              output is found with a decoupled look-back over the slices
//              before it.
#include "wsm_internal.h"

namespace wsm {

constexpr int kSlices = 512;
constexpr int kSliceBits = 15;
constexpr int kPartThreads = 1024;
constexpr int kMaxPpt = 16;                  // pixels per thread (max)
constexpr int kMaxTile = kPartThreads * kMaxPpt;  // 16384 pixels
constexpr int kCompactThreads = 1024;
constexpr int kTileChunk = 2048;             // tiles staged per pass in compact
constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagPrefix = 2ull << 62;
constexpr unsigned long long kValueMask = (1ull << 62) - 1;

struct ReduceLayout {
    int tile;        // pixels per tile (multiple of kPartThreads)
    int ppt;         // pixels per thread
    int64_t ntiles;
    size_t off_keys, off_info, off_status, bytes;
};

static ReduceLayout reduce_layout(int64_t n) {
    ReduceLayout L;
    // Small images get small tiles so that enough blocks run.
    int ppt = 1;
    while (ppt < kMaxPpt && (int64_t)kPartThreads * ppt * 2 * 256 <= n) ppt *= 2;
    L.ppt = ppt;
    L.tile = kPartThreads * ppt;
    L.ntiles = (n + L.tile - 1) / L.tile;
    L.off_keys = 0;
    L.off_info = align_up((size_t)L.ntiles * L.tile * 2, 256);
    L.off_status = align_up(L.off_info + (size_t)kSlices * L.ntiles * 4, 256);
    L.bytes = align_up(L.off_status + kSlices * 8 + 64, 256);
    return L;
}

// ---------------------------------------------------------------------------
template <bool VEC16>
__global__ __launch_bounds__(kPartThreads) void reduce_partition_kernel(
    const uint8_t *__restrict__ rgb, int64_t n, int ppt, int tile,
    int64_t ntiles, uint16_t *__restrict__ keys16,
    uint32_t *__restrict__ info, unsigned long long *__restrict__ status,
    int32_t *__restrict__ err_flag) {
    __shared__ uint32_t hist[kSlices];
    __shared__ uint32_t cursor[kSlices];
    __shared__ uint16_t stage[kMaxTile];
    __shared__ uint32_t wave_tot[kPartThreads / 64];

    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t base = b * (int64_t)tile;
    const int len = (int)((n - base) < tile ? (n - base) : tile);

    if (b == 0) {
        for (int s = tid; s < kSlices; s += kPartThreads) status[s] = 0ull;
        if (tid == 0) *err_flag = 0;
    }
    for (int s = tid; s < kSlices; s += kPartThreads) hist[s] = 0u;
    __syncthreads();

    // Load this thread's ppt consecutive pixels and rank each in its slice.
    uint32_t key[kMaxPpt];
    uint32_t rank[kMaxPpt];
    const int first = tid * ppt;
    if (VEC16 && first + kMaxPpt <= len) {
        // 16 pixels = 48 bytes = three 16-byte loads (tile bases are
        // 48-byte multiples and the image base is 16-byte aligned).
        const uint4 *src = (const uint4 *)(rgb + (base + first) * 3);
        uint4 q0 = src[0], q1 = src[1], q2 = src[2];
        uint32_t w[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y,
                          q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
#pragma unroll
        for (int j = 0; j < kMaxPpt; ++j) {
            const int byte = 3 * j;
            uint32_t r = (w[byte >> 2] >> (8 * (byte & 3))) & 0xFFu;
            uint32_t g = (w[(byte + 1) >> 2] >> (8 * ((byte + 1) & 3))) & 0xFFu;
            uint32_t bl = (w[(byte + 2) >> 2] >> (8 * ((byte + 2) & 3))) & 0xFFu;
            key[j] = (r << 16) | (g << 8) | bl;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kMaxPpt; ++j) {
            key[j] = 0u;
            const int q = first + j;
            if (j < ppt && q < len) {
                const uint8_t *px = rgb + (base + q) * 3;
                key[j] = ((uint32_t)px[0] << 16) | ((uint32_t)px[1] << 8) | (uint32_t)px[2];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kMaxPpt; ++j) {
        rank[j] = 0u;
        if (j < ppt && first + j < len) rank[j] = atomicAdd(&hist[key[j] >> kSliceBits], 1u);
    }
    __syncthreads();

    // Exclusive scan of the 512 slice counts (2 per thread in the first 256).
    uint32_t a0 = 0, a1 = 0;
    if (tid < kSlices / 2) {
        a0 = hist[2 * tid];
        a1 = hist[2 * tid + 1];
    }
    uint32_t v = a0 + a1;
    const int lane = tid & 63, wave = tid >> 6;
    uint32_t incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    if (tid < kSlices / 2) {
        uint32_t wbase = 0;
        for (int w2 = 0; w2 < wave; ++w2) wbase += wave_tot[w2];
        const uint32_t excl = wbase + incl - v;
        cursor[2 * tid] = excl;
        cursor[2 * tid + 1] = excl + a0;
        // (offset << 16 | count) per slice; tile <= 16384 so both fit.
        info[(size_t)(2 * tid) * ntiles + b] = (excl << 16) | a0;
        info[(size_t)(2 * tid + 1) * ntiles + b] = ((excl + a0) << 16) | a1;
    }
    __syncthreads();

#pragma unroll
    for (int j = 0; j < kMaxPpt; ++j) {
        if (j < ppt && first + j < len) {
            const uint32_t k = key[j];
            stage[cursor[k >> kSliceBits] + rank[j]] = (uint16_t)(k & ((1u << kSliceBits) - 1));
        }
    }
    __syncthreads();

    // Coalesced write of the tile's grouped low keys.
    uint16_t *dst = keys16 + base;
    for (int q = tid; q < len; q += kPartThreads) dst[q] = stage[q];
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kCompactThreads) void reduce_compact_kernel(
    const uint16_t *__restrict__ keys16, const uint32_t *__restrict__ info,
    int64_t ntiles, int tile, uint32_t *__restrict__ colors,
    uint32_t *__restrict__ counts, unsigned long long *__restrict__ status,
    int32_t *__restrict__ n_unique, int32_t *__restrict__ err_flag) {
    __shared__ uint32_t hist[1 << kSliceBits];
    __shared__ uint32_t seg_start[kTileChunk + 1];   // prefix of counts in the chunk
    __shared__ uint32_t seg_off[kTileChunk];         // offset within the tile
    __shared__ uint32_t wave_tot[kCompactThreads / 64];
    __shared__ unsigned long long s_excl;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int s = blockIdx.x;

    for (int i = tid; i < (1 << kSliceBits); i += kCompactThreads) hist[i] = 0u;

    for (int64_t c0 = 0; c0 < ntiles; c0 += kTileChunk) {
        const int nt = (int)((ntiles - c0) < kTileChunk ? (ntiles - c0) : kTileChunk);
        __syncthreads();
        // Stage the chunk's (offset, count) words and scan the counts.
        uint32_t cnt0 = 0, cnt1 = 0;
        const int g0 = 2 * tid, g1 = 2 * tid + 1;
        if (g0 < nt) {
            uint32_t w = info[(size_t)s * ntiles + c0 + g0];
            cnt0 = w & 0xFFFFu;
            seg_off[g0] = w >> 16;
        }
        if (g1 < nt) {
            uint32_t w = info[(size_t)s * ntiles + c0 + g1];
            cnt1 = w & 0xFFFFu;
            seg_off[g1] = w >> 16;
        }
        uint32_t v = cnt0 + cnt1, incl = v;
        for (int off = 1; off < 64; off <<= 1) {
            uint32_t o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wave_tot[wave] = incl;
        __syncthreads();
        uint32_t wbase = 0;
        for (int w2 = 0; w2 < wave; ++w2) wbase += wave_tot[w2];
        const uint32_t excl = wbase + incl - v;
        if (g0 < nt) seg_start[g0] = excl;
        if (g1 < nt) seg_start[g1] = excl + cnt0;
        if (tid == kCompactThreads - 1) seg_start[nt] = wbase + incl;
        __syncthreads();
        const uint32_t total = seg_start[nt];
        // Element e of the chunk lives in the tile g with
        // seg_start[g] <= e < seg_start[g+1]; each wave finds g for its first
        // element by bisection and lanes walk forward from there.
        for (uint32_t e0 = (uint32_t)wave * 64; e0 < total; e0 += kCompactThreads) {
            int lo = 0, hi = nt - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (seg_start[mid] <= e0) lo = mid; else hi = mid - 1;
            }
            const uint32_t e = e0 + lane;
            if (e < total) {
                int g = lo;
                while (seg_start[g + 1] <= e) ++g;
                const size_t src = (size_t)(c0 + g) * tile + seg_off[g] + (e - seg_start[g]);
                atomicAdd(&hist[keys16[src]], 1u);
            }
        }
    }
    __syncthreads();

    // Compaction: thread t owns bins [32 t, 32 t + 32).
    constexpr int kBinsPerThread = (1 << kSliceBits) / kCompactThreads;
    uint32_t mine = 0;
#pragma unroll 8
    for (int j = 0; j < kBinsPerThread; ++j) mine += hist[tid * kBinsPerThread + j] != 0u;
    uint32_t incl = mine;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    uint32_t wbase = 0, slice_total = 0;
    for (int w2 = 0; w2 < kCompactThreads / 64; ++w2) {
        if (w2 < wave) wbase += wave_tot[w2];
        slice_total += wave_tot[w2];
    }
    const uint32_t local = wbase + incl - mine;

    // Decoupled look-back for the number of unique colors in slices < s.
    if (tid == 0) {
        unsigned long long excl = 0;
        if (s == 0) {
            __hip_atomic_store(&status[0], kFlagPrefix | slice_total, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&status[s], kFlagAgg | slice_total, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            int j = s - 1;
            const unsigned long long t_start = __builtin_amdgcn_s_memrealtime();
            bool failed = false;
            while (j >= 0) {
                unsigned long long w = __hip_atomic_load(&status[j], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long f = w & ~kValueMask;
                if (f == kFlagPrefix) {
                    excl += w & kValueMask;
                    break;
                } else if (f == kFlagAgg) {
                    excl += w & kValueMask;
                    --j;
                } else {
                    __builtin_amdgcn_s_sleep(1);
                    // Bounded wait (2 s at the 100 MHz constant clock).
                    if (__builtin_amdgcn_s_memrealtime() - t_start > 200000000ull) {
                        failed = true;
                        break;
                    }
                }
            }
            if (failed) {
                atomicOr(err_flag, 1);
                excl = 0;
            }
            __hip_atomic_store(&status[s], kFlagPrefix | (excl + slice_total),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_excl = excl;
        if (s == kSlices - 1) *n_unique = (int32_t)(excl + slice_total);
    }
    __syncthreads();
    if (*(volatile int32_t *)err_flag != 0) {
        if (s == kSlices - 1 && tid == 0) *n_unique = -1;
        return;
    }
    const uint32_t out0 = (uint32_t)s_excl + local;
    uint32_t o = out0;
    for (int j = 0; j < kBinsPerThread; ++j) {
        const int bin = tid * kBinsPerThread + j;
        const uint32_t c = hist[bin];
        if (c != 0u) {
            colors[o] = ((uint32_t)s << kSliceBits) | (uint32_t)bin;
            counts[o] = c;
            ++o;
        }
    }
}

}  // namespace wsm

using namespace wsm;

extern "C" int wsm_reduce_workspace_bytes(int64_t n_pixels, size_t *bytes) {
    if (!bytes || n_pixels < 1 || n_pixels > (int64_t)0xFFFFFFFFll) return WSM_EINVAL;
    *bytes = reduce_layout(n_pixels).bytes;
    return WSM_OK;
}

extern "C" int wsm_reduce_colors(const uint8_t *rgb, int64_t n_pixels, uint32_t *colors,
                                 uint32_t *counts, int64_t cap, int32_t *n_unique,
                                 void *workspace, size_t workspace_bytes, hipStream_t stream) {
    if (!rgb || !colors || !counts || !n_unique || !workspace) return WSM_EINVAL;
    if (n_pixels < 1 || n_pixels > (int64_t)0xFFFFFFFFll) return WSM_EINVAL;
    const int64_t need_cap = n_pixels < (1ll << 24) ? n_pixels : (1ll << 24);
    if (cap < need_cap) return WSM_ENOSPC;
    if (((uintptr_t)workspace & 15u) != 0u) return WSM_EINVAL;
    const ReduceLayout L = reduce_layout(n_pixels);
    if (workspace_bytes < L.bytes) return WSM_ENOSPC;
    char *ws = (char *)workspace;
    uint16_t *keys16 = (uint16_t *)(ws + L.off_keys);
    uint32_t *info = (uint32_t *)(ws + L.off_info);
    unsigned long long *status = (unsigned long long *)(ws + L.off_status);
    int32_t *err = (int32_t *)(ws + L.off_status + kSlices * 8);
    const bool vec = (L.ppt == kMaxPpt) && (((uintptr_t)rgb & 15u) == 0u);
    (void)hipGetLastError();
    timing_before(WSM_KERNEL_REDUCE_PARTITION, stream);
    if (vec)
        reduce_partition_kernel<true><<<dim3((unsigned)L.ntiles), dim3(kPartThreads), 0, stream>>>(
            rgb, n_pixels, L.ppt, L.tile, L.ntiles, keys16, info, status, err);
    else
        reduce_partition_kernel<false><<<dim3((unsigned)L.ntiles), dim3(kPartThreads), 0, stream>>>(
            rgb, n_pixels, L.ppt, L.tile, L.ntiles, keys16, info, status, err);
    timing_after(WSM_KERNEL_REDUCE_PARTITION, stream);
    if (hipGetLastError() != hipSuccess) return WSM_EHIP;
    timing_before(WSM_KERNEL_REDUCE_COMPACT, stream);
    reduce_compact_kernel<<<dim3(kSlices), dim3(kCompactThreads), 0, stream>>>(
        keys16, info, L.ntiles, L.tile, colors, counts, status, n_unique, err);
    timing_after(WSM_KERNEL_REDUCE_COMPACT, stream);
    if (hipGetLastError() != hipSuccess) return WSM_EHIP;
    return WSM_OK;
}
