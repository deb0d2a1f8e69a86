// Block-level building blocks of the sort-means search (Alg. 2) on gfx950,
// shared by the iteration kernel and the pixel-map kernel.
//
// Each block handles a contiguous chunk of points in passes of kPass.  For
// the sort-means scan a point with previous center p walks row p of the
// sorted-neighbour matrix M and stops at the first center t with
// d(c_p,c_t)^2 >= thr(x) = 4 (1 + 2^-16) d(x,c_p)^2.  Within a pass only the
// rows that some point of the pass starts from are ever read, and only up to
// T_p = max thr(x) over those points: every entry past that bound stops every
// scan of the row.  So a block builds, in LDS, exactly that part of M -- row
// p holds the centers t != p with d(c_p,c_t)^2 < T_p, sorted by (distance,
// index) -- and the scans over it visit the same centers, in the same order,
// with the same break, as scans over the full sorted rows.
//
// Rows are built one per wave (wave w takes rows w, w + 16, ...): the wave
// counts the row's entries with a ballot, wave 0 turns the counts into
// offsets, and each wave then writes its rows' entries and sorts them by rank.
// Offsets depend only on the counts, so the layout is deterministic.
#pragma once

#include "wave_ops.h"
#include "wsm_internal.h"

namespace wsm {

constexpr int kCpt = 4;                          // points per thread per pass
constexpr int kPass = kSearchThreads * kCpt;     // points per pass (4096)
constexpr int kMaxSurv = 8192;                   // truncated-row entries per pass

struct RowLists {
    uint32_t thr[kMaxK];   // float bits of T_p (0: no entry can be reached)
    uint32_t len[kMaxK];   // entries of row p
    uint32_t off[kMaxK];   // start of row p in list[]
    int overflow;
    unsigned long long key[kMaxSurv];  // staging: distance bits << 32 | center
    uint8_t list[kMaxSurv];            // the truncated sorted rows
};

__device__ __forceinline__ unsigned long long lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Head flag of a run of equal keys (lane 0 or a different key in the lane
// before).
__device__ __forceinline__ int run_head(int key) {
    const int lane = threadIdx.x & 63;
    const int kp = __shfl_up(key, 1, 64);
    return (lane == 0 || kp != key) ? 1 : 0;
}

__device__ __forceinline__ bool run_tail(int key, bool valid) {
    const int lane = threadIdx.x & 63;
    const int nk = __shfl_down(key, 1, 64);
    const bool nv = __shfl_down((int)valid, 1, 64) != 0;
    return valid && (lane == 63 || !nv || nk != key);
}

// Record the break threshold of one point per lane into L.thr (max per
// row).  All lanes of the wave call it.
__device__ __forceinline__ void add_threshold(RowLists &L, bool valid, int p, float prev) {
    const uint32_t tb = valid ? __float_as_uint(prev * kBreakScale) : 0u;
    const int key = valid ? p : -1;
    const uint32_t mx = wave_seg_max(run_head(key), tb);
    if (run_tail(key, valid) && mx != 0u) atomicMax(&L.thr[p], mx);
}

// Number of entries of row p (centers t != p with d(c_p,c_t)^2 < T).  Called
// by a whole wave; the result is the same in every lane.
__device__ __forceinline__ uint32_t count_row(const float4 *cen, int K, int p, float T) {
    const int lane = threadIdx.x & 63;
    const float4 cp = cen[p];
    uint32_t n = 0;
    for (int c0 = 0; c0 < K; c0 += 64) {
        const int t = c0 + lane;
        bool s = false;
        if (t < K && t != p) {
            const float4 ct = cen[t];
            s = sq_dist(cp.x, cp.y, cp.z, ct.x, ct.y, ct.z) < T;
        }
        n += (uint32_t)__popcll(__ballot(s));
    }
    return n;
}

// Write row p's n entries at `base` and sort them.  Called by a whole wave.
__device__ __forceinline__ void fill_row(RowLists &L, const float4 *cen, int K, int p, float T,
                                         uint32_t n, uint32_t base) {
    const int lane = threadIdx.x & 63;
    const float4 cp = cen[p];
    // the entries (distance bits, center) in center order
    uint32_t w = 0;
    for (int c0 = 0; c0 < K; c0 += 64) {
        const int t = c0 + lane;
        bool s = false;
        float d = 0.f;
        if (t < K && t != p) {
            const float4 ct = cen[t];
            d = sq_dist(cp.x, cp.y, cp.z, ct.x, ct.y, ct.z);
            s = d < T;
        }
        const unsigned long long m = __ballot(s);
        if (s) {
            const uint32_t pos = w + (uint32_t)__popcll(m & lanemask_lt());
            L.key[base + pos] = ((unsigned long long)__float_as_uint(d) << 32) | (unsigned)t;
        }
        w += (uint32_t)__popcll(m);
    }
    // rank sort: entry j's place = number of entries with a smaller key
    // (distance first, then index; keys are distinct)
    for (uint32_t j0 = 0; j0 < n; j0 += 64) {
        const uint32_t j = j0 + lane;
        const unsigned long long kj = j < n ? L.key[base + j] : ~0ull;
        uint32_t r = 0;
        for (uint32_t f = 0; f < n; ++f) r += L.key[base + f] < kj;
        if (j < n) L.list[base + r] = (uint8_t)(kj & 0xFFu);
    }
}

// Build every row whose threshold is set.  Must be called by all threads
// after a barrier that makes L.thr final; ends with a barrier.  Sets
// L.overflow (and builds nothing) if the rows do not fit.
template <int NT>
__device__ void build_row_lists(RowLists &L, const float4 *cen, int K) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // Every lane of the wave stores the same value: no lane-0-only branch at
    // the end of a loop whose body holds cross-lane operations.
    for (int p = wave; p < K; p += NW) {
        const uint32_t tb = L.thr[p];
        const uint32_t n = tb != 0u ? count_row(cen, K, p, __uint_as_float(tb)) : 0u;
        L.len[p] = n;
    }
    __syncthreads();
    if (wave == 0) {
        uint32_t base = 0;
        for (int c0 = 0; c0 < K; c0 += 64) {
            const int p = c0 + lane;
            const uint32_t v = p < K ? L.len[p] : 0u;
            const uint32_t incl = wave_incl_sum(v);
            if (p < K) L.off[p] = base + incl - v;
            base += wave_last_u32(incl);
        }
        L.overflow = base > (uint32_t)kMaxSurv ? 1 : 0;
    }
    __syncthreads();
    if (L.overflow) return;
    for (int p = wave; p < K; p += NW) {
        const uint32_t n = L.len[p];
        if (n != 0u) fill_row(L, cen, K, p, __uint_as_float(L.thr[p]), n, L.off[p]);
    }
    __syncthreads();
}

__device__ __forceinline__ void reset_row_lists(RowLists &L, int K) {
    for (int c = threadIdx.x; c < K; c += blockDim.x) L.thr[c] = 0u;
}

// Sort-means scan over the truncated row of p.
__device__ __forceinline__ int sm_scan_lists(float x, float y, float z, int p,
                                             const float4 *cen, const RowLists &L,
                                             float &best_d, uint32_t &ev) {
    const float4 cp = cen[p];
    const float prev = sq_dist(x, y, z, cp.x, cp.y, cp.z);
    const float thr = prev * kBreakScale;
    float bd = prev;
    int best = p;
    ev += 1;
    const uint32_t o = L.off[p], n = L.len[p];
    for (uint32_t j = 0; j < n; ++j) {
        const int t = L.list[o + j];
        const float4 ct = cen[t];
        const float dpt = sq_dist(cp.x, cp.y, cp.z, ct.x, ct.y, ct.z);
        if (dpt >= thr) break;
        const float d = sq_dist(x, y, z, ct.x, ct.y, ct.z);
        ev += 1;
        if (better_center(d, bd, t, best, p)) {
            bd = d;
            best = t;
        }
    }
    best_d = bd;
    return best;
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

// Block sums in a fixed order: waves reduce with DPP, wave totals are added
// in wave order.  Result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum_f64(double v, double *scr) {
    v = wave_sum_f64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 63) scr[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) s += scr[w];
    return s;
}

template <int NT>
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long *scr) {
    v = wave_sum_u64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 63) scr[wave] = v;
    __syncthreads();
    unsigned long long s = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) s += scr[w];
    return s;
}

}  // namespace wsm
