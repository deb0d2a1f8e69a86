// Data reduction of the WSM quantizer (Sec. 2, "data sampling" and "sample
// weighting"): the unique 24-bit colors of an image with their pixel counts,
// emitted in ascending key order.
//
// Two kernels, both staging their hot data in LDS:
//   partition  one block per tile of up to 16384 pixels.  Each pixel's key
//              R<<16 | G<<8 | B is split into a slice (top 9 bits, 512
//              slices) and a 15-bit low key.  An LDS histogram of the tile's
//              slices gives every pixel a rank; the low keys are written out
//              grouped by slice (a tile-local counting sort), 2 bytes per
//              pixel with 16-byte stores, together with an (offset, count)
//              word per (slice, tile).  The blocks of one XCD take
//              consecutive tiles (xcd_tile).
//   compact    one block per slice.  Each wave takes the slice's segments
//              in a set of tiles (one (offset, count) word per lane), lays
//              them end to end as a list of 16-byte pieces and deals the
//              pieces out to its lanes, 64 per round and kRoundsInFlight
//              rounds' loads in flight at once, so that nearly every lane
//              counts 8 of the slice's keys per round into a 2^15-bin LDS
//              histogram however long or short the segments are; the
//              non-empty bins are compacted in
//              ascending order, and the slice's place in the output comes
//              from a decoupled look-back over the slices before it, 64
//              predecessors per step.
#include <mutex>

#include "wave_ops.h"
#include "wsm_internal.h"

namespace wsm {

constexpr int kSlices = 512;
constexpr int kSliceBits = 15;
constexpr int kPartThreads = 1024;
constexpr int kMaxPpt = 16;                       // pixels per thread (max)
constexpr int kMaxTile = kPartThreads * kMaxPpt;  // 16384 pixels
constexpr int kCompactThreads = 1024;
constexpr int kCompactWaves = kCompactThreads / 64;
constexpr int kRoundsInFlight = 2;                // 16-byte loads in flight per lane
constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagPrefix = 2ull << 62;
constexpr unsigned long long kValueMask = (1ull << 62) - 1;

struct ReduceLayout {
    int tile;        // pixels per tile (multiple of kPartThreads)
    int ppt;         // pixels per thread
    int64_t ntiles;
    size_t off_keys, off_info, off_status, bytes;
};

constexpr ReduceLayout reduce_layout(int64_t n) {
    ReduceLayout L{};
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

// Tile of partition block blk.  Workgroups are dealt to the 8 XCDs in turn,
// so the blocks of one XCD (equal blk mod 8) take a consecutive run of tiles:
// each line of a slice's (offset, count) words is then written whole by one
// XCD's L2.  The grid is ntiles rounded up to a multiple of 8; a block left
// without a tile returns ntiles.
__device__ __forceinline__ int64_t xcd_tile(int64_t blk, int64_t ntiles) {
    const int64_t x = blk & 7, j = blk >> 3;
    const int64_t q = ntiles >> 3, r = ntiles & 7;
    const int64_t cnt = q + (x < r ? 1 : 0);
    return j < cnt ? x * q + (x < r ? x : r) + j : ntiles;
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
    __shared__ __align__(16) uint16_t stage[kMaxTile];
    __shared__ uint32_t wave_tot[kPartThreads / 64];

    const int tid = threadIdx.x;
    const int64_t b = xcd_tile(blockIdx.x, ntiles);
    if (b >= ntiles) return;
    const int64_t base = b * (int64_t)tile;
    const int len = (int)((n - base) < tile ? (n - base) : tile);

    if (b == 0) {
        for (int s = tid; s < kSlices; s += kPartThreads) status[s] = 0ull;
        if (tid == 0) *err_flag = 0;
    }
    for (int s = tid; s < kSlices; s += kPartThreads) hist[s] = 0u;

    // Load this thread's ppt consecutive pixels.
    uint32_t key[kMaxPpt];
    uint32_t rank[kMaxPpt];
    const int first = tid * ppt;
    if (VEC16 && first + kMaxPpt <= len) {
        // 16 pixels = 48 bytes = three 16-byte loads (tile bases are
        // 48-byte multiples and the image base is 16-byte aligned).
        const uint4 *src = (const uint4 *)(rgb + (base + first) * 3);
        const uint4 q0 = src[0], q1 = src[1], q2 = src[2];
        const uint32_t w[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y,
                                q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
#pragma unroll
        for (int j = 0; j < kMaxPpt; ++j) {
            const int byte = 3 * j;
            const uint32_t r = (w[byte >> 2] >> (8 * (byte & 3))) & 0xFFu;
            const uint32_t g = (w[(byte + 1) >> 2] >> (8 * ((byte + 1) & 3))) & 0xFFu;
            const uint32_t bl = (w[(byte + 2) >> 2] >> (8 * ((byte + 2) & 3))) & 0xFFu;
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
    __syncthreads();
    // Rank every pixel within its slice.
#pragma unroll
    for (int j = 0; j < kMaxPpt; ++j) {
        rank[j] = 0u;
        if (j < ppt && first + j < len) rank[j] = atomicAdd(&hist[key[j] >> kSliceBits], 1u);
    }
    __syncthreads();

    // Exclusive scan of the 512 slice counts (2 per thread in the first 256).
    const int lane = tid & 63, wave = tid >> 6;
    uint32_t a0 = 0, a1 = 0;
    if (tid < kSlices / 2) {
        a0 = hist[2 * tid];
        a1 = hist[2 * tid + 1];
    }
    const uint32_t v = a0 + a1;
    const uint32_t incl = wave_incl_sum(v);
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

    // Write the tile's grouped low keys: 8 keys (16 bytes) per store.
    uint16_t *dst = keys16 + base;
    const int full = len & ~7;
    for (int q = tid * 8; q < full; q += kPartThreads * 8)
        *(uint4 *)(dst + q) = *(const uint4 *)(stage + q);
    for (int q = full + tid; q < len; q += kPartThreads) dst[q] = stage[q];
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kCompactThreads) void reduce_compact_kernel(
    const uint16_t *__restrict__ keys16, const uint32_t *__restrict__ info,
    int64_t ntiles, int tile, uint32_t *__restrict__ colors,
    uint32_t *__restrict__ counts, unsigned long long *__restrict__ status,
    int32_t *__restrict__ n_unique, int32_t *__restrict__ err_flag) {
    __shared__ __align__(16) uint32_t hist[1 << kSliceBits];
    // per wave: the rounds in flight' marks of where the lanes' pieces start
    __shared__ uint8_t marks[kCompactWaves][64 * kRoundsInFlight];
    __shared__ uint32_t wave_tot[kCompactThreads / 64];
    __shared__ unsigned long long s_excl;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int s = blockIdx.x;

    // Lane l of wave w holds the word of tile c0 + kCompactWaves l + w of the
    // tiles c0 .. c0 + 1023 (one pass of the block), so every wave has work
    // however few tiles there are.  The first pass's words are requested
    // before the histogram is cleared.
    auto word_of = [&](int64_t c0) -> uint32_t {
        const int64_t tw = c0 + kCompactWaves * lane + wave;
        return tw < ntiles ? info[(size_t)s * ntiles + tw] : 0u;
    };
    uint32_t w = word_of(0);
    for (int i = tid * 4; i < (1 << kSliceBits); i += kCompactThreads * 4)
        *(uint4 *)(hist + i) = make_uint4(0u, 0u, 0u, 0u);
    for (int i = lane; i < 64 * kRoundsInFlight; i += 64) marks[wave][i] = 0u;
    __syncthreads();

    // Histogram.  The lane's segment [st, st + n) (key indices relative to
    // the pass's first key: at most 1024 tiles of 16384 keys, so 32 bits)
    // covers the 16-byte pieces st / 8 .. (st + n - 1) / 8; the wave lists
    // all its lanes' pieces in lane order (an exclusive sum gives each lane
    // where its own start) and takes them in rounds of 64, lane j piece
    // q0 + j.  The lanes whose first piece falls in the rounds in flight
    // mark it with 1 + their lane; a running maximum over the wave, carried
    // from round to round, then gives each piece its segment.  A wave's LDS
    // operations take effect in issue order, and signal fences keep the
    // compiler from reordering them.
    for (int64_t c0 = 0; c0 < ntiles; c0 += 64 * kCompactWaves) {
        if (c0 != 0) w = word_of(c0);
        const uint16_t *kb = keys16 + (size_t)c0 * tile;
        const uint32_t st = (uint32_t)(kCompactWaves * lane + wave) * (uint32_t)tile + (w >> 16);
        const uint32_t n = w & 0xFFFFu;
        const uint32_t pieces = n ? ((st + n - 1u) >> 3) - (st >> 3) + 1u : 0u;
        const uint32_t incl = wave_incl_sum(pieces);
        const uint32_t excl = incl - pieces;
        const uint32_t total = wave_last_u32(incl);
        uint32_t carry = 0u;
        for (uint32_t q0 = 0; q0 < total; q0 += 64 * kRoundsInFlight) {  // wave-uniform
            const bool mark = pieces != 0u && excl >= q0 && excl < q0 + 64 * kRoundsInFlight;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (mark) marks[wave][excl - q0] = (uint8_t)(lane + 1);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            uint32_t hq[kRoundsInFlight];
#pragma unroll
            for (int r = 0; r < kRoundsInFlight; ++r) hq[r] = marks[wave][64 * r + lane];
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (mark) marks[wave][excl - q0] = 0u;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            uint32_t a[kRoundsInFlight], lo[kRoundsInFlight], hi[kRoundsInFlight];
            uint4 v[kRoundsInFlight];
#pragma unroll
            for (int r = 0; r < kRoundsInFlight; ++r) {
                uint32_t o1 = wave_incl_max(hq[r]);
                o1 = o1 > carry ? o1 : carry;
                carry = wave_last_u32(o1);
                const int o = o1 ? (int)o1 - 1 : 0;
                const uint32_t st_o = (uint32_t)__shfl((int)st, o, 64);
                const uint32_t n_o = (uint32_t)__shfl((int)n, o, 64);
                const uint32_t ex_o = (uint32_t)__shfl((int)excl, o, 64);
                const uint32_t q = q0 + 64 * r + lane;
                const bool act = q < total;
                a[r] = ((st_o >> 3) + (q - ex_o)) << 3;
                lo[r] = act ? st_o : 0u;
                hi[r] = act ? st_o + n_o : 0u;
                v[r] = act ? *(const uint4 *)(kb + a[r]) : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int r = 0; r < kRoundsInFlight; ++r) {
                const uint32_t wd[4] = {v[r].x, v[r].y, v[r].z, v[r].w};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t pos = a[r] + e;
                    if (pos >= lo[r] && pos < hi[r])
                        atomicAdd(&hist[(wd[e >> 1] >> (16 * (e & 1))) & 0xFFFFu], 1u);
                }
            }
        }
    }
    __syncthreads();

    // Compaction: wave w owns bins [2048 w, 2048 w + 2048); lane l visits
    // bins 2048 w + 64 j + l, so LDS reads are conflict-free and the
    // non-empty bins come out in ascending order with a ballot per step.
    constexpr int kBinsPerWave = (1 << kSliceBits) / (kCompactThreads / 64);
    const uint32_t *wb = hist + wave * kBinsPerWave;
    uint32_t mine = 0;
#pragma unroll 8
    for (int j = 0; j < kBinsPerWave; j += 64) mine += __popcll(__ballot(wb[j + lane] != 0u));
    if (lane == 0) wave_tot[wave] = mine;
    __syncthreads();
    uint32_t wbase = 0, slice_total = 0;
    for (int w2 = 0; w2 < kCompactThreads / 64; ++w2) {
        if (w2 < wave) wbase += wave_tot[w2];
        slice_total += wave_tot[w2];
    }
    const uint32_t local = wbase;

    // Decoupled look-back for the number of unique colors in slices < s:
    // the first wave reads 64 predecessors' words per step.
    if (wave == 0) {
        if (lane == 0)
            __hip_atomic_store(&status[s], (s == 0 ? kFlagPrefix : kFlagAgg) | slice_total,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long excl = 0;
        bool failed = false;
        int j = s - 1;
        const unsigned long long t_start = __builtin_amdgcn_s_memrealtime();
        while (j >= 0) {
            // Every lane loads (a clamped index keeps the address valid);
            // lanes past slice 0 then act as a zero prefix.
            const int idx = j - lane;
            const unsigned long long ld = __hip_atomic_load(
                &status[idx >= 0 ? idx : 0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long wv = idx >= 0 ? ld : kFlagPrefix;
            const unsigned long long f = wv & ~kValueMask;
            const unsigned long long pre = __ballot(f == kFlagPrefix);
            const unsigned long long none = __ballot(f == 0ull);
            // lanes up to and including the nearest prefix must all be ready
            const int stop = pre ? __ffsll((long long)pre) - 1 : 63;
            const unsigned long long need = stop == 63 ? ~0ull : ((2ull << stop) - 1ull);
            if (none & need) {
                __builtin_amdgcn_s_sleep(1);
                // Bounded wait (2 s at the 100 MHz constant clock).
                if (__builtin_amdgcn_s_memrealtime() - t_start > 200000000ull) {
                    failed = true;
                    break;
                }
                continue;
            }
            const unsigned long long val = (lane <= stop) ? (wv & kValueMask) : 0ull;
            const unsigned long long tot = wave_sum_u64(val);
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)tot, 63);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(tot >> 32), 63);
            excl += ((unsigned long long)hi << 32) | lo;
            if (pre) break;
            j -= 64;
        }
        if (failed) {
            if (lane == 0) atomicOr(err_flag, 1);
            excl = 0;
        }
        if (lane == 0) {
            if (s != 0)
                __hip_atomic_store(&status[s], kFlagPrefix | (excl + slice_total),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_excl = excl;
            if (s == kSlices - 1) *n_unique = (int32_t)(excl + slice_total);
        }
    }
    __syncthreads();
    if (*(volatile int32_t *)err_flag != 0) {
        if (s == kSlices - 1 && tid == 0) *n_unique = -1;
        return;
    }
    uint32_t o = (uint32_t)s_excl + local;
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int j = 0; j < kBinsPerWave; j += 64 * 4) {
        uint32_t c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = wb[j + 64 * u + lane];  // reads issued together
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int bin = wave * kBinsPerWave + j + 64 * u + lane;
            const unsigned long long m = __ballot(c[u] != 0u);
            if (c[u] != 0u) {
                const uint32_t pos = o + (uint32_t)__popcll(m & below);
                colors[pos] = ((uint32_t)s << kSliceBits) | (uint32_t)bin;
                counts[pos] = c[u];
            }
            o += (uint32_t)__popcll(m);
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

static int reduce_launch(const uint8_t *rgb, int64_t n_pixels, uint32_t *colors,
                         uint32_t *counts, int32_t *n_unique, void *workspace,
                         const ReduceLayout &L, hipStream_t stream);

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
    return reduce_launch(rgb, n_pixels, colors, counts, n_unique, workspace, L, stream);
}

static int reduce_launch(const uint8_t *rgb, int64_t n_pixels, uint32_t *colors,
                         uint32_t *counts, int32_t *n_unique, void *workspace,
                         const ReduceLayout &L, hipStream_t stream) {
    char *ws = (char *)workspace;
    uint16_t *keys16 = (uint16_t *)(ws + L.off_keys);
    uint32_t *info = (uint32_t *)(ws + L.off_info);
    unsigned long long *status = (unsigned long long *)(ws + L.off_status);
    int32_t *err = (int32_t *)(ws + L.off_status + kSlices * 8);
    const bool vec = (L.ppt == kMaxPpt) && (((uintptr_t)rgb & 15u) == 0u);
    (void)hipGetLastError();
    if (vec)
        WSM_LAUNCH(WSM_KERNEL_REDUCE_PARTITION, reduce_partition_kernel<true>,
                   dim3((unsigned)((L.ntiles + 7) & ~7ll)), dim3(kPartThreads), stream, rgb, n_pixels, L.ppt,
                   L.tile, L.ntiles, keys16, info, status, err);
    else
        WSM_LAUNCH(WSM_KERNEL_REDUCE_PARTITION, reduce_partition_kernel<false>,
                   dim3((unsigned)((L.ntiles + 7) & ~7ll)), dim3(kPartThreads), stream, rgb, n_pixels, L.ppt,
                   L.tile, L.ntiles, keys16, info, status, err);
    if (hipGetLastError() != hipSuccess) return WSM_EHIP;
    WSM_LAUNCH(WSM_KERNEL_REDUCE_COMPACT, reduce_compact_kernel, dim3(kSlices),
               dim3(kCompactThreads), stream, (const uint16_t *)keys16, (const uint32_t *)info,
               L.ntiles, L.tile, colors, counts, status, n_unique, err);
    if (hipGetLastError() != hipSuccess) return WSM_EHIP;
    return WSM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free variant of wsm_reduce_colors: its workspace is the
// file-scope device array `scratch`, sized for the largest image it takes
// (WSM_STATIC_MAX_PIXELS).  Every GPU the library runs on holds its own
// copy until the process ends.  In host code `scratch` names a host-side
// stand-in, so its device address is looked up (hipGetSymbolAddress) the
// first time the entry point runs on a device, with that device current,
// and kept per device; only that address is passed to the kernels.  The
// partition kernel clears the look-back flags and the error word it uses,
// so nothing left by an earlier call needs clearing.
constexpr size_t kScratchBytes = reduce_layout(WSM_STATIC_MAX_PIXELS).bytes;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device.
int scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) {
        (void)hipGetLastError();
        return WSM_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return WSM_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return WSM_OK;
}

}  // namespace

extern "C" int wsm_reduce_colors_static(const uint8_t *rgb, int64_t n_pixels, uint32_t *colors,
                                        uint32_t *counts, int64_t cap, int32_t *n_unique,
                                        hipStream_t stream) {
    if (!rgb || !colors || !counts || !n_unique) return WSM_EINVAL;
    if (n_pixels < 1) return WSM_EINVAL;
    if (n_pixels > (int64_t)WSM_STATIC_MAX_PIXELS) return WSM_ENOSPC;
    const int64_t need_cap = n_pixels < (1ll << 24) ? n_pixels : (1ll << 24);
    if (cap < need_cap) return WSM_ENOSPC;
    const ReduceLayout L = reduce_layout(n_pixels);
    if (L.bytes > kScratchBytes) return WSM_ENOSPC;
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != WSM_OK) return rc;
    return reduce_launch(rgb, n_pixels, colors, counts, n_unique, ws, L, stream);
}
