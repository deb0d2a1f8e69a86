// Wave-level (64-lane) scans and reductions on gfx950 built from DPP lane
// moves (row_shr within rows of 16 lanes, row_bcast15 / row_bcast31 across
// rows).  DPP moves are VALU operations, so a full 64-lane scan is a chain of
// six short VALU steps instead of six LDS round trips through ds_bpermute.
//
// All functions must be called by every lane of the wave (no divergence).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wsm {

// DPP controls (GFX9 encoding).
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
    const uint32_t lo = dpp_u32<CTRL>((uint32_t)v);
    const uint32_t hi = dpp_u32<CTRL>((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    return __longlong_as_double((long long)dpp_u64<CTRL>((unsigned long long)__double_as_longlong(v)));
}

// Whether the lane receiving a move with control CTRL combines it, for an
// inclusive scan in lane order.
template <int CTRL>
__device__ __forceinline__ bool dpp_takes(int lane) {
    const int rl = lane & 15;
    if (CTRL == kDppRowShr1) return rl >= 1;
    if (CTRL == kDppRowShr2) return rl >= 2;
    if (CTRL == kDppRowShr4) return rl >= 4;
    if (CTRL == kDppRowShr8) return rl >= 8;
    if (CTRL == kDppRowBcast15) return (lane >> 4) & 1;   // rows 1 and 3
    return lane >= 32;                                     // row_bcast31: rows 2, 3
}

// Inclusive prefix sum over the wave.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
    const int lane = threadIdx.x & 63;
    uint32_t t;
    t = dpp_u32<kDppRowShr1>(v);
    if (dpp_takes<kDppRowShr1>(lane)) v += t;
    t = dpp_u32<kDppRowShr2>(v);
    if (dpp_takes<kDppRowShr2>(lane)) v += t;
    t = dpp_u32<kDppRowShr4>(v);
    if (dpp_takes<kDppRowShr4>(lane)) v += t;
    t = dpp_u32<kDppRowShr8>(v);
    if (dpp_takes<kDppRowShr8>(lane)) v += t;
    t = dpp_u32<kDppRowBcast15>(v);
    if (dpp_takes<kDppRowBcast15>(lane)) v += t;
    t = dpp_u32<kDppRowBcast31>(v);
    if (dpp_takes<kDppRowBcast31>(lane)) v += t;
    return v;
}

// One step of a segmented inclusive scan: (f, v) of this lane combined with
// the moved (f', v') of a preceding lane: v += v' unless a segment starts in
// between (f set), and f |= f'.
template <int CTRL>
__device__ __forceinline__ void seg_step_sum2(int lane, int &f, unsigned long long &a,
                                              unsigned long long &b) {
    const int tf = dpp_i32<CTRL>(f);
    const unsigned long long ta = dpp_u64<CTRL>(a);
    const unsigned long long tb = dpp_u64<CTRL>(b);
    if (dpp_takes<CTRL>(lane)) {
        if (!f) {
            a += ta;
            b += tb;
        }
        f |= tf;
    }
}

// Segmented inclusive sums of two 64-bit values; a segment starts at lanes
// with head != 0.  The last lane of each segment ends with the segment sum.
__device__ __forceinline__ void wave_seg_sum2(int head, unsigned long long &a,
                                              unsigned long long &b) {
    const int lane = threadIdx.x & 63;
    int f = head;
    seg_step_sum2<kDppRowShr1>(lane, f, a, b);
    seg_step_sum2<kDppRowShr2>(lane, f, a, b);
    seg_step_sum2<kDppRowShr4>(lane, f, a, b);
    seg_step_sum2<kDppRowShr8>(lane, f, a, b);
    seg_step_sum2<kDppRowBcast15>(lane, f, a, b);
    seg_step_sum2<kDppRowBcast31>(lane, f, a, b);
}

// Inclusive maximum over the wave, in lane order.
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
    const int lane = threadIdx.x & 63;
    uint32_t t;
    t = dpp_u32<kDppRowShr1>(v);
    if (dpp_takes<kDppRowShr1>(lane)) v = v > t ? v : t;
    t = dpp_u32<kDppRowShr2>(v);
    if (dpp_takes<kDppRowShr2>(lane)) v = v > t ? v : t;
    t = dpp_u32<kDppRowShr4>(v);
    if (dpp_takes<kDppRowShr4>(lane)) v = v > t ? v : t;
    t = dpp_u32<kDppRowShr8>(v);
    if (dpp_takes<kDppRowShr8>(lane)) v = v > t ? v : t;
    t = dpp_u32<kDppRowBcast15>(v);
    if (dpp_takes<kDppRowBcast15>(lane)) v = v > t ? v : t;
    t = dpp_u32<kDppRowBcast31>(v);
    if (dpp_takes<kDppRowBcast31>(lane)) v = v > t ? v : t;
    return v;
}

// Sum over the wave in a fixed order; the result is valid in lane 63.
__device__ __forceinline__ double wave_sum_f64(double v) {
    const int lane = threadIdx.x & 63;
    double t;
    t = dpp_f64<kDppRowShr1>(v);
    if (dpp_takes<kDppRowShr1>(lane)) v += t;
    t = dpp_f64<kDppRowShr2>(v);
    if (dpp_takes<kDppRowShr2>(lane)) v += t;
    t = dpp_f64<kDppRowShr4>(v);
    if (dpp_takes<kDppRowShr4>(lane)) v += t;
    t = dpp_f64<kDppRowShr8>(v);
    if (dpp_takes<kDppRowShr8>(lane)) v += t;
    t = dpp_f64<kDppRowBcast15>(v);
    if (dpp_takes<kDppRowBcast15>(lane)) v += t;
    t = dpp_f64<kDppRowBcast31>(v);
    if (dpp_takes<kDppRowBcast31>(lane)) v += t;
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    const int lane = threadIdx.x & 63;
    unsigned long long t;
    t = dpp_u64<kDppRowShr1>(v);
    if (dpp_takes<kDppRowShr1>(lane)) v += t;
    t = dpp_u64<kDppRowShr2>(v);
    if (dpp_takes<kDppRowShr2>(lane)) v += t;
    t = dpp_u64<kDppRowShr4>(v);
    if (dpp_takes<kDppRowShr4>(lane)) v += t;
    t = dpp_u64<kDppRowShr8>(v);
    if (dpp_takes<kDppRowShr8>(lane)) v += t;
    t = dpp_u64<kDppRowBcast15>(v);
    if (dpp_takes<kDppRowBcast15>(lane)) v += t;
    t = dpp_u64<kDppRowBcast31>(v);
    if (dpp_takes<kDppRowBcast31>(lane)) v += t;
    return v;
}

// Minimum over the wave; the result is valid in lane 63.
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
    const int lane = threadIdx.x & 63;
    unsigned long long t;
    t = dpp_u64<kDppRowShr1>(v);
    if (dpp_takes<kDppRowShr1>(lane) && t < v) v = t;
    t = dpp_u64<kDppRowShr2>(v);
    if (dpp_takes<kDppRowShr2>(lane) && t < v) v = t;
    t = dpp_u64<kDppRowShr4>(v);
    if (dpp_takes<kDppRowShr4>(lane) && t < v) v = t;
    t = dpp_u64<kDppRowShr8>(v);
    if (dpp_takes<kDppRowShr8>(lane) && t < v) v = t;
    t = dpp_u64<kDppRowBcast15>(v);
    if (dpp_takes<kDppRowBcast15>(lane) && t < v) v = t;
    t = dpp_u64<kDppRowBcast31>(v);
    if (dpp_takes<kDppRowBcast31>(lane) && t < v) v = t;
    return v;
}

// Value of lane 63 broadcast to the wave (scalar reads).
__device__ __forceinline__ unsigned long long wave_last_u64(unsigned long long v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

// Value of lane 63 broadcast to the wave (scalar read).
__device__ __forceinline__ uint32_t wave_last_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

}  // namespace wsm
