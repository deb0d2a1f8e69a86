// Internal definitions shared by the gfx950 kernels of the WSM library:
// state layout, launch constants and the small device helpers every step
// uses.  Nothing here is part of the C ABI (see include/wsm.h).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/wsm.h"

namespace wsm {

constexpr int kMaxK = WSM_MAX_K;
constexpr int kHistory = WSM_HISTORY;
constexpr int kMaxGrid = 2048;          // upper bound on search-kernel blocks
constexpr int kSearchThreads = 1024;    // threads per search block (16 waves)
constexpr int kRowThreads = 256;        // threads of the single-block final update
constexpr int kSortThreads = 1024;      // threads per rows block (one row of M each)
constexpr uint32_t kMagic = 0x574D5331u;

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Measurement hook (timing.hip).  timing_claim hands out the next pair of
// events when a caller attached events to this kernel kind; WSM_LAUNCH then
// launches through hipExtLaunchKernelGGL, which records them at the
// kernel's start and end.
bool timing_claim(int kind, hipEvent_t *begin, hipEvent_t *end);

#define WSM_LAUNCH(KIND, KERNEL, GRID, BLOCK, STREAM, ...)                                   \
    do {                                                                                     \
        hipEvent_t wsm_tb_, wsm_te_;                                                         \
        if (::wsm::timing_claim((KIND), &wsm_tb_, &wsm_te_))                                 \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, wsm_tb_, wsm_te_, 0,       \
                                  __VA_ARGS__);                                              \
        else                                                                                 \
            KERNEL<<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);                                 \
    } while (0)

// ---------------------------------------------------------------------------
// Per-iteration record.  Two copies live in the state header: the kernels of
// call-relative step i read copy (i & 1) and write copy ((i + 1) & 1), so no
// block ever reads a record another block of the same launch is writing.
struct Record {
    int32_t iters;      // iterations completed (t of the last update)
    int32_t converged;  // the Sec. 3.2 criterion (or SSE == 0) has fired
    int32_t err;        // device-side error bits
    int32_t mode;       // how the centers after the update are searched (kMode*)
    double sse_last;    // SSE_t of the last completed iteration
    double pad2;
};
static_assert(sizeof(Record) == 32, "record layout");

struct Header {
    uint32_t magic;
    int32_t k;
    int32_t points;
    int32_t grid;
    int64_t n_points;
    int64_t n_pixels;
    int32_t wild;       // the initial palette has a coordinate outside [0, 256)
    int32_t pad;
    uint64_t reserved[3];
    Record rec[2];      // bytes 64..127
    int32_t info[4];    // bytes 128..143: public copy {iters, converged, err, 0}
};
static_assert(offsetof(Header, rec) == 64, "header layout");
static_assert(offsetof(Header, info) == 128, "header layout");

// State layout (byte offsets).  Sizes do not depend on k; only the
// membership array at the end depends on the number of points.
constexpr size_t kOffHeader = 0;
constexpr size_t kOffPalette = 256;                                   // float4[2][256]
constexpr size_t kOffPal64 = kOffPalette + 2 * kMaxK * 16;            // double4[2][256]
// Center totals: three slots (filled, read, cleared by step parity mod 3),
// each with kTotCopies copies of u64[256][4].  A block adds into the copy of
// its physical index mod kTotCopies; workgroups are dealt to the 8 XCDs in
// turn, so each copy takes the atomics of one XCD and no line moves between
// the XCDs' L2 caches.  Readers add the copies (exact integers).
constexpr int kTotCopies = 8;
constexpr size_t kTotCopy = (size_t)kMaxK * 4;                        // u64 words per copy
constexpr size_t kTotSlot = kTotCopies * kTotCopy;                     // u64 words per slot
constexpr size_t kOffTotals = kOffPal64 + 2 * kMaxK * 32;             // u64[3][kTotCopies][256][4]
constexpr size_t kOffSsePart = kOffTotals + 3 * kTotSlot * 8;         // double[2][kMaxGrid]
constexpr size_t kOffEvalPart = kOffSsePart + 2 * kMaxGrid * 8;       // u64[2][kMaxGrid]
constexpr size_t kOffSseHist = kOffEvalPart + 2 * kMaxGrid * 8;       // double[kHistory]
constexpr size_t kOffEvalHist = kOffSseHist + kHistory * 8;           // int64[kHistory]
constexpr size_t kOffMapPart = kOffEvalHist + kHistory * 8;           // double[kMaxGrid]
constexpr size_t kOffRows = align_up(kOffMapPart + kMaxGrid * 8, 256);  // u8[256][256]
constexpr int kRowDist = 64;  // leading entries of each row whose distances are kept
constexpr size_t kOffRowDist = kOffRows + (size_t)kMaxK * kMaxK;  // float[256][kRowDist]
constexpr size_t kOffMembership = kOffRowDist + (size_t)kMaxK * kRowDist * 4;

inline size_t state_bytes_for(int64_t n_points) {
    return kOffMembership + align_up((size_t)n_points, 256);
}

// Typed device view of a state block.
struct StateView {
    Header *hdr;
    float4 *pal;          // [2][256]
    double4 *pal64;       // [2][256]: the same palettes in float64 (pal is their rounding)
    unsigned long long *totals;  // [3][256][4]
    double *sse_part;     // [2][kMaxGrid]
    unsigned long long *eval_part;  // [2][kMaxGrid]
    double *sse_hist;
    long long *eval_hist;
    double *map_part;     // [kMaxGrid]
    uint8_t *rows;        // [256][256]: sorted neighbour rows (M without self)
    float *rowd;          // [256][kRowDist]: d(c_p, c_t)^2 of the first entries of row p
    uint8_t *m;           // [n_points]
};

inline StateView make_view(void *state) {
    char *b = (char *)state;
    StateView v;
    v.hdr = (Header *)(b + kOffHeader);
    v.pal = (float4 *)(b + kOffPalette);
    v.pal64 = (double4 *)(b + kOffPal64);
    v.totals = (unsigned long long *)(b + kOffTotals);
    v.sse_part = (double *)(b + kOffSsePart);
    v.eval_part = (unsigned long long *)(b + kOffEvalPart);
    v.sse_hist = (double *)(b + kOffSseHist);
    v.eval_hist = (long long *)(b + kOffEvalHist);
    v.map_part = (double *)(b + kOffMapPart);
    v.rows = (uint8_t *)(b + kOffRows);
    v.rowd = (float *)(b + kOffRowDist);
    v.m = (uint8_t *)(b + kOffMembership);
    return v;
}

// Points a state is bound to: unique colors + counts, or raw pixels.
struct Points {
    const uint32_t *colors;
    const uint32_t *counts;
    const uint8_t *rgb;
    int64_t n;
    int32_t is_pixels;
};

// ---------------------------------------------------------------------------
// Squared RGB distance (Eq. 1 uses ||x - c||^2).  One fixed expression is
// used everywhere -- for the center table, its row sort, the break test and
// the point distances -- so a distance recomputed in the scan is bit-equal
// to the one the row was sorted by.  The library is built with
// -ffp-contract=off; the two fused multiply-adds are explicit.
__device__ __forceinline__ float sq_dist(float ax, float ay, float az,
                                         float bx, float by, float bz) {
    float dx = ax - bx;
    float dy = ay - by;
    float dz = az - bz;
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// Break test of the sort-means scan: stop at center t once
// d(c_p, c_t)^2 >= 4 d(x, c_p)^2 (triangle inequality, Sec. 2).  The float32
// test is made conservative by a factor 1 + 2^-16 so that rounding in the
// three squared distances can never skip a center that the float32 full
// search would choose (the rounding error of each is below 2^-21 relative).
constexpr float kBreakScale = 4.0f * (1.0f + 1.0f / 65536.0f);

// Tie key (dist, k != p, k): on equal distance keep the previous center p,
// otherwise prefer the lower index.  t is never p.
__device__ __forceinline__ bool better_center(float d, float best_d, int t,
                                              int best, int p) {
    return d < best_d || (d == best_d && best != p && t < best);
}

__device__ __forceinline__ void unpack_key(uint32_t key, float &r, float &g,
                                           float &b) {
    r = (float)((key >> 16) & 0xFFu);
    g = (float)((key >> 8) & 0xFFu);
    b = (float)(key & 0xFFu);
}

// ---------------------------------------------------------------------------
// Float64 decisions.  A center is the weighted mean S_k / W_k of exact
// integer sums (Alg. 2, last loop); its float64 value is the correctly
// rounded mean and its float32 value the rounding of that.  The searches
// run in float32; each point's float32 choice is kept only when it is
// certainly the choice float64 arithmetic makes (the smallest key
// (d, k != p, k) over all centers with d the float64 squared distance), and
// the rest are decided again in float64 over all centers.  How a set of
// centers is searched:
constexpr int kModeExact = 0;    // every coordinate an integer: float32 distances are exact
constexpr int kModeCertify = 1;  // coordinates in [0, 256): certified float32, rest in float64
constexpr int kModeResolve = 2;  // any other center: every choice made in float64
constexpr float kNoSkip = 3.402823466e38f;  // no row entry skipped / no second distance

// Squared RGB distance in float64, summed left to right (the library is
// built with -ffp-contract=off, so nothing is fused).
__device__ __forceinline__ double sq_dist64(double ax, double ay, double az, double bx,
                                            double by, double bz) {
    const double dx = ax - bx;
    const double dy = ay - by;
    const double dz = az - bz;
    return dx * dx + dy * dy + dz * dz;
}

// Bound on |d32 - D|, d32 a squared distance computed by sq_dist from
// float32-rounded centers (coordinates in [0, 256)) and D the exact distance
// from the float64 centers.  Each coordinate difference is off by at most
// 3 * 2^-17 (two center roundings of at most 2^-17 and the float32
// subtraction), which moves D by at most 2 sqrt(3 D) 3 * 2^-17 < 2^-13 sqrt(D)
// plus second-order terms; the three float32 roundings of the sum add at most
// 3 * 2^-24 d.  Each term carries a margin of at least 1.5x, and the constant
// covers distances near zero.  The square root is the hardware one (within a
// few ulp), which the margins absorb.
__device__ __forceinline__ float f32_err(float d) {
    return d * 0x1p-21f + __builtin_amdgcn_sqrtf(d) * 0x1p-13f + 0x1p-22f;
}

// The same bound without the square root: distances between colors and
// centers in [0, 256)^3 are below 3 * 256^2, so sqrt(d) < 444 and
// 2^-13 sqrt(d) + 2^-22 < 2^-4.
__device__ __forceinline__ float f32_err_max(float d) { return d * 0x1p-21f + 0x1p-4f; }

// Whether a float32 sort-means (or full) scan's choice is certainly the
// float64 one.  bd: distance to the chosen center; s2: second smallest
// distance among the evaluated centers (the previous center included;
// kNoSkip if none); prev: distance to the previous center; dj: d(c_p, c_t)^2
// of the first row entry the scan skipped (kNoSkip if it skipped none).
//   (i) every other evaluated center is farther than the chosen one by more
//       than both error bounds;
//  (ii) every skipped center t has d(c_p, c_t)^2 >= dj (the row is sorted),
//       so by the triangle inequality its distance from x is at least
//       (sqrt(dj) - sqrt(d(x, c_p)^2))^2, which must exceed the chosen
//       distance.  The chosen distance is at most the previous center's, so
//       it suffices that (sqrt(dj') - sqrt(prev'))^2 > prev' (1 + 2^-16),
//       primes marking the bounds taken on the safe side; that holds when
//       dj' > 4 prev' (1 + 2^-15).  Otherwise the chosen distance itself is
//       compared (the factor 1 + 2^-16 covers the float32 square roots and
//       the subtraction).
// Each test is first tried with f32_err_max, which needs no square root
// and decides almost every point; certified_exact, out of line, redoes the
// tests with f32_err only for the rest.
__device__ __noinline__ bool certified_exact(float bd, float s2, float prev, float dj);

__device__ __forceinline__ bool certified(float bd, float s2, float prev, float dj) {
    const bool i_fast = s2 - f32_err_max(s2) > bd + f32_err_max(bd);
    const bool ii_fast =
        !(dj < kNoSkip) || dj - f32_err_max(dj) > 4.0f * (prev + f32_err_max(prev)) * (1.0f + 0x1p-15f);
    return (i_fast && ii_fast) || certified_exact(bd, s2, prev, dj);
}

__device__ __noinline__ bool certified_exact(float bd, float s2, float prev, float dj) {
    if (!(s2 - f32_err(s2) > bd + f32_err(bd))) return false;
    if (dj < kNoSkip) {
        const float eb = bd + f32_err(bd);
        const float r = __builtin_amdgcn_sqrtf(fmaxf(dj - f32_err(dj), 0.0f)) -
                        __builtin_amdgcn_sqrtf(prev + f32_err(prev));
        if (!(r > 0.0f && r * r > eb * (1.0f + 0x1p-16f))) return false;
    }
    return true;
}

// Mode of a set of centers (kMode*), from flags each thread collects over
// its share of them: kFlagNonInt for a coordinate that is not an integer,
// kFlagWild for one outside [0, 256) (or not a number).
constexpr int kFlagNonInt = 1;
constexpr int kFlagWild = 2;

__device__ __forceinline__ int coord_flags(double v) {
    if (!(v >= 0.0 && v < 256.0)) return kFlagWild;
    return v != floor(v) ? kFlagNonInt : 0;
}

__device__ __forceinline__ int center_flags(double4 c) {
    return coord_flags(c.x) | coord_flags(c.y) | coord_flags(c.z);
}

// Block-wide vote on the flags (a barrier: all threads call it).
__device__ __forceinline__ int block_mode(int flags) {
    const int wild = __syncthreads_or(flags & kFlagWild);
    const int nonint = __syncthreads_or(flags & kFlagNonInt);
    return wild ? kModeResolve : nonint ? kModeCertify : kModeExact;
}

}  // namespace wsm
