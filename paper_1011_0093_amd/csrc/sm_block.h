// Building blocks of the sort-means search (Alg. 2) on gfx950, shared by the
// iteration kernels and the pixel-map kernel.
//
// The sorted-neighbour matrix M (Sec. 2): row p lists the centers t != p in
// ascending (d(c_p, c_t)^2, t) order -- the row's first entry, p itself, is
// left out, since the scan starts from the second one.  It is built once per
// set of centers (sort_row, one block per row) and kept in device memory as
// K rows of kRowStride bytes, with the distances of each row's first
// kRowDist entries; a search block copies the rows (for K >= kDeferMinK
// only their first kRowPrefix entries and those distances) into LDS.  (For
// K <= kFusedMaxK every search block sorts the rows itself, with a row
// table: entry j of row p as (c_t, d(c_p, c_t)^2).)  A scan compares
// d(c_p, c_t)^2 recomputed from the centers in LDS, or the stored value,
// with the same expression the rows were sorted by, so the break test sees
// bit-equal values.
//
// For K < kDeferMinK a lane scans its own point's row, kScanBatch entries
// at a time (sm_scan, or sm_scan_tab over a row table).  For K >=
// kDeferMinK each lane scans the first kLaneHead entries of its point's row
// and a wave then takes the rest of its 64 points' row heads together, with
// the entries dealt out evenly over the lanes (sm_scan_flat), and the rare
// scans that go past the head are finished by the whole wave
// (sm_finish_wave), so that no lane holds its wave.
#pragma once

#include "wave_ops.h"
#include "wsm_internal.h"

namespace wsm {

constexpr int kCpt = 2;                          // points per thread of a search block's first pass
constexpr int kPass = 4096;                      // points per block and pass of the default grid rule
constexpr int kRowStride = kMaxK;                // bytes per row of M in device memory
constexpr int kScanBatch = 8;                    // row entries fetched per scan step
static_assert(kScanBatch == 8, "a scan batch is one 8-byte word of a row, read aligned");
static_assert(kMaxK % kScanBatch == 0, "a batched full scan stays inside the center table");
constexpr int kRowPrefix = 64;                   // row head scanned flat (in LDS when scans defer)
constexpr int kLaneHead = 16;                    // entries of the flat scan a lane takes itself
static_assert(kRowPrefix == kRowDist, "the stored distances cover the LDS row prefix");
constexpr int kDeferCap = 1024;                  // deferred scans per block
constexpr int kDeferBatch = 8;                   // deferred scans a wave fetches rows for at once
constexpr int kDeferMinK = 33;                   // smallest K whose search scans flat
constexpr int kFusedMaxK = 32;                   // largest K sorted inside the search block
static_assert(kDeferMinK == kFusedMaxK + 1, "the launches past the fused kernel scan flat");

// LDS row stride for K centers: K - 1 entries rounded up to 16 bytes.
__host__ __device__ constexpr int lds_row_stride(int K) { return ((K - 1) + 15) / 16 * 16; }

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

// Sort row p of M for the K centers in LDS and write it to `row` (device
// memory).  keys (u64) and rank (u32) are LDS scratch of kMaxK entries.  The
// key of center t is (distance bits, t): distances are non-negative, so
// their bit patterns order like the values, and the keys are distinct.  The
// rank of each key is counted by NT / kMaxK threads over slices of the
// others.  If drow is not null, the distances of the first kRowDist entries
// are written to it as well.  All NT threads call it; it starts with a
// barrier, so consecutive calls may reuse the scratch.
template <int NT>
__device__ void sort_row(const float4 *cen, int K, int p, unsigned long long *__restrict__ keys,
                         uint32_t *rank, uint8_t *__restrict__ row, float *__restrict__ drow) {
    static_assert(NT % kMaxK == 0, "block size");
    constexpr int Q = NT / kMaxK;
    constexpr int span = kMaxK / Q;
    const int tid = threadIdx.x;
    __syncthreads();
    const float4 cp = cen[p];
    for (int t = tid; t < kMaxK; t += NT) {
        unsigned long long kt = ~0ull;
        if (t < K && t != p) {
            const float4 ct = cen[t];
            kt = ((unsigned long long)__float_as_uint(sq_dist(cp.x, cp.y, cp.z, ct.x, ct.y, ct.z))
                  << 32) | (unsigned)t;
        }
        keys[t] = kt;
        rank[t] = 0u;
    }
    __syncthreads();
    const int t = tid % kMaxK, q = tid / kMaxK;
    if (t < K && t != p) {
        const unsigned long long kt = keys[t];
        const int u0 = q * span;
        const int u1 = (u0 + span) < K ? (u0 + span) : K;
        // eight keys per step, read as four 16-byte words; keys past K hold
        // the largest value and never count
        const ulonglong2 *k2 = (const ulonglong2 *)keys;
        uint32_t r = 0;
        for (int u = u0; u < u1; u += 8) {
            const ulonglong2 a = k2[u / 2], b = k2[u / 2 + 1], c = k2[u / 2 + 2], d = k2[u / 2 + 3];
            r += (uint32_t)(a.x < kt) + (uint32_t)(a.y < kt) + (uint32_t)(b.x < kt) +
                 (uint32_t)(b.y < kt) + (uint32_t)(c.x < kt) + (uint32_t)(c.y < kt) +
                 (uint32_t)(d.x < kt) + (uint32_t)(d.y < kt);
        }
        if (Q == 1)
            rank[t] = r;
        else
            atomicAdd(&rank[t], r);
    }
    __syncthreads();
    for (int c = tid; c < K; c += NT) {
        if (c != p) {
            const uint32_t rk = rank[c];
            row[rk] = (uint8_t)c;
            if (drow && rk < (uint32_t)kRowDist)
                drow[rk] = __uint_as_float((uint32_t)(keys[c] >> 32));
        }
    }
}

// Copy the K rows of M (device layout, kRowStride bytes per row) into LDS
// rows of lds_row_stride(K) bytes: fetch_rows issues a thread's loads into
// registers, store_rows writes them to LDS.  All threads of the block call
// both.
template <int NT>
struct RowRegs {
    static constexpr int kRegs = (kMaxK * kRowStride / 16 + NT - 1) / NT;
    uint4 v[kRegs];
};

// LDS row stride: PREFIX rows hold the first kRowPrefix entries only, other
// rows all K - 1.
template <bool PREFIX>
__device__ __forceinline__ int lds_rows_stride(int K) {
    return PREFIX ? kRowPrefix : lds_row_stride(K);
}

// 16-byte pieces per thread that fetch_rows / store_rows move
template <int NT, bool PREFIX>
constexpr int row_regs() {
    return PREFIX ? (kMaxK * kRowPrefix / 16 + NT - 1) / NT : RowRegs<NT>::kRegs;
}

template <int NT, bool PREFIX = false>
__device__ __forceinline__ void fetch_rows(const uint8_t *__restrict__ M, int K, RowRegs<NT> &R) {
    const int per_row = lds_rows_stride<PREFIX>(K) / 16;
    const int nq = K * per_row;
#pragma unroll
    for (int u = 0; u < row_regs<NT, PREFIX>(); ++u) {
        const int q = threadIdx.x + u * NT;
        R.v[u] = make_uint4(0u, 0u, 0u, 0u);
        if (q < nq) {
            const int r = q / per_row, c = q - r * per_row;
            R.v[u] = *(const uint4 *)(M + (size_t)r * kRowStride + c * 16);
        }
    }
}

template <int NT, bool PREFIX = false>
__device__ __forceinline__ void store_rows(const RowRegs<NT> &R, int K, uint8_t *Ms) {
    const int rs = lds_rows_stride<PREFIX>(K);
    const int per_row = rs / 16;
    const int nq = K * per_row;
#pragma unroll
    for (int u = 0; u < row_regs<NT, PREFIX>(); ++u) {
        const int q = threadIdx.x + u * NT;
        if (q < nq) {
            const int r = q / per_row, c = q - r * per_row;
            *(uint4 *)(Ms + r * rs + c * 16) = R.v[u];
        }
    }
}

template <int NT>
__device__ __forceinline__ void load_rows(const uint8_t *__restrict__ M, int K, uint8_t *Ms) {
    RowRegs<NT> R;
    fetch_rows<NT>(M, K, R);
    store_rows<NT>(R, K, Ms);
}

// Where a scan reads row p: the LDS copy (stride rs) holds its first `len`
// entries; entries from `len` on are read from device memory (g, the row of
// M in the state).
struct RowView {
    const uint8_t *lds;
    const uint8_t *g;
    int len;
};

// Sort-means scan (Alg. 2, inner loop) of point x from its previous center
// p over the LDS copy of M: starting from d(x, c_p), centers are taken in row
// order until the first t with d(c_p, c_t)^2 >= thr = 4 (1 + 2^-16) d(x, c_p)^2.
//
// sm_scan_range takes the row entries [j, min(j_end, K - 1)) in batches of
// kScanBatch (one 8-byte read of the row, the center reads issued together,
// then the entries taken in order; distances computed past the stop are
// discarded) and returns whether the scan has ended (stop found or row
// exhausted); j is left at the next batch.  Reads past the row's K - 1
// entries stay inside the row (its strides are multiples of 16) and the
// center table.  s2 tracks the second smallest evaluated distance (the
// previous center's included); dj is set to d(c_p, c_t)^2 of the entry the
// scan stops at (left alone when the row runs out).
__device__ __forceinline__ bool sm_scan_range(float x, float y, float z, int p, int K,
                                              const float4 *cen, const RowView &row, float thr,
                                              int &j, int j_end, float &bd, int &best,
                                              float &s2, float &dj, uint32_t &ev) {
    const float4 cp = cen[p];
    const int n = K - 1;
    const int jm = j_end < n ? j_end : n;
    for (; j < jm; j += kScanBatch) {
        const uint2 w8 = j + kScanBatch <= row.len ? *(const uint2 *)(row.lds + j)
                                                   : *(const uint2 *)(row.g + j);
        float dpt[kScanBatch], d[kScanBatch];
        int t[kScanBatch];
#pragma unroll
        for (int e = 0; e < kScanBatch; ++e) {
            t[e] = ((e < 4 ? w8.x : w8.y) >> (8 * (e & 3))) & 0xFFu;
            const float3 ct = *(const float3 *)(cen + t[e]);  // the 4th lane is unused
            dpt[e] = sq_dist(cp.x, cp.y, cp.z, ct.x, ct.y, ct.z);
            d[e] = sq_dist(x, y, z, ct.x, ct.y, ct.z);
        }
        bool stop = false;
#pragma unroll
        for (int e = 0; e < kScanBatch; ++e) {
            if (!stop) {
                if (j + e >= n || dpt[e] >= thr) {
                    stop = true;
                    if (j + e < n) dj = dpt[e];
                } else {
                    ev += 1;
                    s2 = fminf(s2, fmaxf(d[e], bd));
                    if (better_center(d[e], bd, t[e], best, p)) {
                        bd = d[e];
                        best = t[e];
                    }
                }
            }
        }
        if (stop) return true;
    }
    return j >= n;
}

// The whole scan of one point over its row in LDS, in one loop: the start
// at the previous center, then the row in batches as in sm_scan_range.
// Besides the choice and its distance it returns what certified() needs:
// the previous center's distance, the second smallest evaluated distance and
// the first skipped entry's center distance (kNoSkip if none was skipped).
__device__ __forceinline__ int sm_scan(float x, float y, float z, int p, int K,
                                       const float4 *cen, const uint8_t *Ms, int rs,
                                       float &best_d, float &prev_out, float &s2_out,
                                       float &dj_out, uint32_t &ev) {
    const float4 cp = cen[p];
    const float prev = sq_dist(x, y, z, cp.x, cp.y, cp.z);
    const float thr = prev * kBreakScale;
    float bd = prev;
    float s2 = kNoSkip, dj = kNoSkip;
    int best = p;
    ev += 1;
    const uint8_t *row = Ms + p * rs;
    const int n = K - 1;
    for (int j = 0; j < n; j += kScanBatch) {
        const uint2 w8 = *(const uint2 *)(row + j);
        float dpt[kScanBatch], d[kScanBatch];
        int t[kScanBatch];
#pragma unroll
        for (int e = 0; e < kScanBatch; ++e) {
            t[e] = ((e < 4 ? w8.x : w8.y) >> (8 * (e & 3))) & 0xFFu;
            const float3 ct = *(const float3 *)(cen + t[e]);  // the 4th lane is unused
            dpt[e] = sq_dist(cp.x, cp.y, cp.z, ct.x, ct.y, ct.z);
            d[e] = sq_dist(x, y, z, ct.x, ct.y, ct.z);
        }
        bool stop = false;
#pragma unroll
        for (int e = 0; e < kScanBatch; ++e) {
            if (!stop) {
                if (j + e >= n || dpt[e] >= thr) {
                    stop = true;
                    if (j + e < n) dj = dpt[e];
                } else {
                    ev += 1;
                    s2 = fminf(s2, fmaxf(d[e], bd));
                    if (better_center(d[e], bd, t[e], best, p)) {
                        bd = d[e];
                        best = t[e];
                    }
                }
            }
        }
        if (stop) break;
    }
    best_d = bd;
    prev_out = prev;
    s2_out = s2;
    dj_out = dj;
    return best;
}

// sm_scan over a row table: entry j of row p is also kept as the float4
// (c_t, d(c_p, c_t)^2) in Tb[p * ts + j] (t = the row's entry j), so a batch
// of kScanBatch entries takes one round of LDS reads -- the row's 8 indices
// and the 8 table entries, whose addresses are all known -- instead of the
// center reads waiting for the indices.  The stored d(c_p, c_t)^2 is the
// value the rows were sorted by.  Same results as sm_scan.  Reads past the
// row's K - 1 entries stay inside the row and its table row (ts and rs are
// at least K - 1 rounded up to kScanBatch); their values are not used.
__device__ __forceinline__ int sm_scan_tab(float x, float y, float z, int p, int K,
                                           const float4 *cen, const uint8_t *Ms, int rs,
                                           const float4 *Tb, int ts, float &best_d,
                                           float &prev_out, float &s2_out, float &dj_out,
                                           uint32_t &ev) {
    const float4 cp = cen[p];
    const float prev = sq_dist(x, y, z, cp.x, cp.y, cp.z);
    const float thr = prev * kBreakScale;
    float bd = prev;
    float s2 = kNoSkip, dj = kNoSkip;
    int best = p;
    ev += 1;
    const uint8_t *row = Ms + p * rs;
    const float4 *tr = Tb + p * ts;
    const int n = K - 1;
    for (int j = 0; j < n; j += kScanBatch) {
        const uint2 w8 = *(const uint2 *)(row + j);
        float4 ce[kScanBatch];
#pragma unroll
        for (int e = 0; e < kScanBatch; ++e) ce[e] = tr[j + e];
        float d[kScanBatch];
        int t[kScanBatch];
#pragma unroll
        for (int e = 0; e < kScanBatch; ++e) {
            t[e] = ((e < 4 ? w8.x : w8.y) >> (8 * (e & 3))) & 0xFFu;
            d[e] = sq_dist(x, y, z, ce[e].x, ce[e].y, ce[e].z);
        }
        bool stop = false;
#pragma unroll
        for (int e = 0; e < kScanBatch; ++e) {
            if (!stop) {
                if (j + e >= n || ce[e].w >= thr) {
                    stop = true;
                    if (j + e < n) dj = ce[e].w;
                } else {
                    ev += 1;
                    s2 = fminf(s2, fmaxf(d[e], bd));
                    if (better_center(d[e], bd, t[e], best, p)) {
                        bd = d[e];
                        best = t[e];
                    }
                }
            }
        }
        if (stop) break;
    }
    best_d = bd;
    prev_out = prev;
    s2_out = s2;
    dj_out = dj;
    return best;
}

// Order key of a candidate under the tie rule (dist, k != p, k): smaller is
// better.  Distances are non-negative, so their bits order like the values.
__device__ __forceinline__ unsigned long long scan_key(float d, int t, int p) {
    return ((unsigned long long)__float_as_uint(d) << 32) | (unsigned)(t == p ? 0 : 256 + t);
}

// Distance part of a scan_key.
__device__ __forceinline__ float key_dist(unsigned long long k) {
    return __uint_as_float((uint32_t)(k >> 32));
}

// Whether two float32 distances of one point may be in the other order, or
// equal, in float64: their difference is within the sum of their error
// bounds (f32_err is increasing, so twice the larger bound covers it).  A
// scan that meets such a pair with its best center cannot certify its
// choice; it reports the near tie as s2 = bd (no near tie: s2 = kNoSkip),
// which certified() rejects.
__device__ __forceinline__ bool near_pair(float a, float b) {
    const float hi = fmaxf(a, b), lo = fminf(a, b);
    return hi - lo <= 2.0f * f32_err(hi);
}

// The rest of one point's scan, from row entry j, by the whole wave: lane l
// takes entry j + l, the stop is the first entry (in row order) at or past
// the threshold, and the entries before it are reduced with scan_key.  Every
// argument but t_first is the same in all lanes, and all 64 lanes must call
// it; t_first is row entry j + lane, loaded by the caller (any value where
// j + lane >= K - 1).  The results (bd, best, s2 as near_pair reports it --
// s2 < kNoSkip on entry means a near tie was seen before -- the stop entry's
// center distance dj, kNoSkip if the row runs out, and the evaluations made)
// are the same in all lanes.  A near tie with the final best is caught
// either within the 64-entry step that holds that best (every other entry
// of the step against the step's minimum) or when a step's minimum meets
// the best of the entries before it.
__device__ __forceinline__ void sm_finish_wave(float x, float y, float z, int p, int K,
                                               const float4 *cen, const RowView &row, float thr,
                                               int j, int t_first, float &bd, int &best,
                                               float &s2, float &dj, uint32_t &evals) {
    const int lane = threadIdx.x & 63;
    const int n = K - 1;
    const float4 cp = cen[p];
    unsigned long long bk = scan_key(bd, best, p);
    bool near = s2 < kNoSkip;
    uint32_t sev = 0;
    dj = kNoSkip;
    for (int jb = j; jb < n; jb += 64) {
        const int jj = jb + lane;
        const bool in = jj < n;
        const int t = !in ? 0 : jb == j ? t_first : jj < row.len ? row.lds[jj] : row.g[jj];
        const float4 ct = cen[t];
        const float dpt = sq_dist(cp.x, cp.y, cp.z, ct.x, ct.y, ct.z);
        const float d = sq_dist(x, y, z, ct.x, ct.y, ct.z);
        const unsigned long long smask = __ballot(!in || dpt >= thr);
        const int first = smask != 0ull ? __builtin_ctzll(smask) : 64;
        const bool ok = lane < first;
        sev += (uint32_t)__popcll(__ballot(ok));
        const unsigned long long kl = ok ? scan_key(d, t, p) : ~0ull;
        const unsigned long long m1 = wave_last_u64(wave_min_u64(kl));
        if (m1 != ~0ull) {  // wave-uniform
            const float dm = key_dist(m1);
            const bool ln = ok && kl != m1 && near_pair(d, dm);
            near = near || __ballot(ln) != 0ull || near_pair(dm, key_dist(bk));
            bk = m1 < bk ? m1 : bk;
        }
        if (first < 64) {
            const float dstop = __shfl(dpt, first, 64);
            if (jb + first < n) dj = dstop;
            break;
        }
    }
    bd = key_dist(bk);
    best = (bk & 0x100ull) ? (int)(bk & 0xFFull) : p;
    s2 = near ? bd : kNoSkip;
    evals = sev;
}

// LDS scratch of one wave for sm_scan_flat.
struct FlatScratch {
    float4 pt[64];               // lane l: the point (x, y, z) and, as int bits, the
                                 // offset of its pair q's row entry: p * kRowPrefix - first pair
    unsigned long long bk[64];   // lane l: smallest scan_key so far
    uint32_t near[64];           // lane l: a near tie with its best was seen
    uint8_t head[64];            // pair q0 + k of the current round: 1 + the lane whose
                                 // pairs start there, else 0
};

// Sort-means scans of a wave's points (lane l: the point with color `key` and
// previous center p, if valid) over the first L = min(K - 1, kRowPrefix)
// entries of their rows, with the entries spread evenly over the lanes
// rather than each lane scanning its own row: scan lengths differ a lot
// within a wave, and a wave runs as long as its longest lane.
//   Row p is ascending in d(c_p, c_t)^2, so the entries before the break are
// the first n, n = the number of stored distances Dd[p][.] below the
// threshold (a binary search).  The first kLaneHead of them (most scans
// end there) each lane evaluates itself, in row order.  The wave lists the
// remaining (point, entry) pairs in
// lane order and takes them in rounds of 64, lane l pair q0 + l of round q0;
// it finds the pair's point from the marks of where each point's pairs start
// (the lanes whose first pair falls in the round write them; a running
// maximum over the wave spreads them), and folds the pair's scan_key into
// that point's LDS minimum (a
// row never lists its own center, so the pair's key is that of a center
// other than the previous one).
//   The result is the sequential scan's: bd, best, evaluations 1 + n, and
// `more` when the break lies past entry L - 1 and the row goes on (the scan
// then continues from entry L with threshold thr).  It also returns the
// previous center's distance, s2 as near_pair reports it (each pair's key
// goes into the point's minimum, and is compared with the minimum it meets
// there: of the final minimum and any key near it, the later of the two to
// arrive meets the other or a key between them) and the center distance dj
// of the stop entry (kNoSkip if the row runs out; unset with `more`).  Ms holds rows of kRowPrefix entries.  All
// 64 lanes call it.  Lanes of one wave exchange data through LDS here; LDS
// operations of a wave take effect in issue order, and signal fences keep
// the compiler from reordering them.
__device__ __forceinline__ void sm_scan_flat(bool valid, uint32_t key, int p, int K,
                                             const float4 *cen, const uint8_t *Ms,
                                             const float *Dd, FlatScratch &fs, float &thr,
                                             float &prev_out, float &bd, float &s2, float &dj,
                                             int &best, uint32_t &ev, bool &more) {
    const int lane = threadIdx.x & 63;
    const int L = K - 1 < kRowPrefix ? K - 1 : kRowPrefix;
    const int pp = valid ? p : 0;
    float x, y, z;
    unpack_key(key, x, y, z);
    const float4 cp = cen[pp];
    const float prev = sq_dist(x, y, z, cp.x, cp.y, cp.z);
    thr = prev * kBreakScale;
    const float *dr = Dd + pp * kRowPrefix;
    int n = 0;
#pragma unroll
    for (int step = kRowPrefix; step > 0; step >>= 1)
        if (n + step <= L && dr[n + step - 1] < thr) n += step;
    if (!valid) n = 0;
    more = valid && n == L && L < K - 1;
    dj = n < L ? dr[n] : kNoSkip;
    prev_out = prev;
    // The first n1 = min(n, kLaneHead) pairs by the lane itself, in row
    // order, as in sm_scan: the best (tie rule of better_center, the same
    // order as scan_key's) and the second smallest distance s2 among the
    // evaluated centers, the previous one included.  Its near-tie flag is
    // then whether s2 is near the best: near_pair is monotone in the larger
    // distance, so that covers every evaluated center.
    const int n1 = n < kLaneHead ? n : kLaneHead;
    unsigned long long bk;
    bool nr;
    {
        constexpr int kWords = kLaneHead < 8 ? 1 : kLaneHead / 8;  // 8-entry words of the row head
        uint2 w8[kWords];
#pragma unroll
        for (int u = 0; u < kWords; ++u) w8[u] = ((const uint2 *)(Ms + pp * kRowPrefix))[u];
        float hb = prev, hs2 = kNoSkip;
        int hbest = pp;
#pragma unroll
        for (int e = 0; e < kLaneHead; ++e) {
            if (e < n1) {
                const uint2 w = w8[e >> 3];
                const int t = (int)((((e & 7) < 4 ? w.x : w.y) >> (8 * (e & 3))) & 0xFFu);
                const float3 ct = *(const float3 *)(cen + t);  // the 4th lane is unused
                const float d = sq_dist(x, y, z, ct.x, ct.y, ct.z);
                hs2 = fminf(hs2, fmaxf(d, hb));
                if (better_center(d, hb, t, hbest, pp)) {
                    hb = d;
                    hbest = t;
                }
            }
        }
        bk = scan_key(hb, hbest, pp);
        nr = hs2 < kNoSkip && near_pair(hs2, hb);
    }
    // The rest of the pairs, entries n1 .. n - 1, dealt over the wave.
    const int n2 = n - n1;
    const uint32_t incl = wave_incl_sum((uint32_t)n2);
    const int excl = (int)incl - n2;
    const int total = (int)wave_last_u32(incl);
    if (total == 0) {  // wave-uniform: every scan ended within its lane's part
        bd = key_dist(bk);
        s2 = nr ? bd : kNoSkip;
        best = (bk & 0x100ull) ? (int)(bk & 0xFFull) : pp;
        if (valid) ev += 1u + (uint32_t)n;
        return;
    }
    fs.head[lane] = 0u;
    fs.pt[lane] = make_float4(x, y, z, __int_as_float(pp * kRowPrefix + n1 - excl));
    fs.bk[lane] = bk;
    fs.near[lane] = nr ? 1u : 0u;
    uint32_t carry = 0u;
    // A pair's key is compared with the minimum it met one iteration late,
    // so the wait for the returned value overlaps the next iteration's LDS
    // reads.
    int pend_o = -1;
    unsigned long long pend_old = 0ull, pend_kq = 0ull;
    for (int q0 = 0; q0 < total; q0 += 64) {  // wave-uniform
        const int q = q0 + lane;
        const bool act = q < total;
        // this round's marks: written, read, and cleared again by their
        // writers (a wave's LDS operations take effect in issue order)
        const bool mark = n2 > 0 && excl >= q0 && excl < q0 + 64;
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (mark) fs.head[excl - q0] = (uint8_t)(lane + 1);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const uint32_t hq = act ? (uint32_t)fs.head[lane] : 0u;
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (mark) fs.head[excl - q0] = 0u;
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (pend_o >= 0 && near_pair(key_dist(pend_kq), key_dist(pend_old))) fs.near[pend_o] = 1u;
        pend_o = -1;
        uint32_t o1 = wave_incl_max(hq);
        o1 = o1 > carry ? o1 : carry;
        carry = wave_last_u32(o1);
        if (act) {
            const int o = (int)o1 - 1;
            const float4 po = fs.pt[o];
            const int t = Ms[__float_as_int(po.w) + q];
            const float4 ct = cen[t];
            pend_kq = scan_key(sq_dist(po.x, po.y, po.z, ct.x, ct.y, ct.z), t, -1);
            pend_old = atomicMin(&fs.bk[o], pend_kq);
            pend_o = o;
        }
    }
    if (pend_o >= 0 && near_pair(key_dist(pend_kq), key_dist(pend_old))) fs.near[pend_o] = 1u;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const unsigned long long b = fs.bk[lane];
    bd = key_dist(b);
    s2 = fs.near[lane] != 0u ? bd : kNoSkip;
    best = (b & 0x100ull) ? (int)(b & 0xFFull) : pp;
    if (valid) ev += 1u + (uint32_t)n;
}

// The float64 choice for the point with color key and previous center p:
// the smallest key (d, k != p, k) over all K centers, d = sq_dist64 from the
// float64 centers cen64 (LDS).  The whole wave searches, lane l taking the
// centers l, l + 64, ...; key and p are the same in all 64 lanes, which all
// call it.  Returns the center and its float64 distance (in all lanes).
// Rare, so kept out of line (the result comes back in registers).
struct Choice64 {
    double d64;
    int best;
};

__device__ __noinline__ Choice64 resolve_wave(uint32_t key, int p, int K, const double4 *cen64) {
    const int lane = threadIdx.x & 63;
    const double x = (double)((key >> 16) & 0xFFu);
    const double y = (double)((key >> 8) & 0xFFu);
    const double z = (double)(key & 0xFFu);
    unsigned long long bk = ~0ull;  // the lane's smallest distance (bits; d >= 0)
    int bt = 0;
    for (int k = lane; k < K; k += 64) {
        const double4 c = cen64[k];
        const unsigned long long db =
            (unsigned long long)__double_as_longlong(sq_dist64(x, y, z, c.x, c.y, c.z));
        // k ascends within a lane: an equal distance wins only for k == p
        if (db < bk || (db == bk && k == p)) {
            bk = db;
            bt = k;
        }
    }
    const unsigned long long dmin = wave_last_u64(wave_min_u64(bk));
    const unsigned long long tie = bk == dmin ? (bt == p ? 0ull : 1ull + (unsigned)bt) : ~0ull;
    const unsigned long long tmin = wave_last_u64(wave_min_u64(tie));
    Choice64 c;
    c.d64 = __longlong_as_double((long long)dmin);
    c.best = tmin == 0ull ? p : (int)(tmin - 1ull);
    return c;
}

// Float64 decisions of a wave's points (see kMode*).  Lane l holds the
// float32 scan's result for its point: `fin` (a point whose scan is complete
// here), its color key, previous center p, the chosen center best with
// distance bd, and s2, prev, dj as for certified().  Every point whose
// choice is not certified is decided again by resolve_wave, one point at a
// time by the whole wave.  Returns the float64 distance from the point to
// its (possibly new) best center, 0 where fin is false.  All 64 lanes call
// it.
__device__ __forceinline__ double decide64(bool fin, uint32_t key, int p, int K, int mode,
                                           const double4 *cen64, int &best, float bd, float s2,
                                           float prev, float dj) {
    const int lane = threadIdx.x & 63;
    const bool need = fin && (mode == kModeResolve ||
                              (mode == kModeCertify && !certified(bd, s2, prev, dj)));
    unsigned long long amb = __ballot(need);
    double d64 = 0.0;
    while (amb != 0ull) {  // wave-uniform
        const int l = __builtin_ctzll(amb);
        amb &= amb - 1ull;
        const uint32_t kl = (uint32_t)__shfl((int)key, l, 64);
        const int pl = __shfl(p, l, 64);
        const Choice64 c = resolve_wave(kl, pl, K, cen64);
        if (lane == l) {
            best = c.best;
            d64 = c.d64;
        }
    }
    if (fin && !need) {
        if (mode == kModeExact) {
            d64 = (double)bd;  // integer centers and colors: the float32 distance is exact
        } else {
            const double4 c = cen64[best];
            d64 = sq_dist64((double)((key >> 16) & 0xFFu), (double)((key >> 8) & 0xFFu),
                            (double)(key & 0xFFu), c.x, c.y, c.z);
        }
    }
    return d64;
}

// Queue of a block's deferred scans (LDS): points whose scan goes past the
// row head, with the state of the scan so far.
struct DeferQueue {
    uint32_t n;
    uint32_t idx[kDeferCap];    // point index
    uint32_t key[kDeferCap];    // its color and count
    uint32_t cnt[kDeferCap];
    uint32_t bd[kDeferCap];     // best distance so far (float bits)
    uint32_t s2[kDeferCap];     // second smallest distance so far (float bits)
    uint32_t pjb[kDeferCap];    // next entry << 16 | previous center << 8 | best center
};
struct NoQueue {};

// How a search launch holds M in LDS and scans it:
//   kVarFirst: whole rows (a call's first step: the full scan on a fresh
//              state, else sm_scan);
//   kVarLane:  whole rows, sm_scan (the batched form's steps for K <
//              kDeferMinK);
//   kVarDefer: K >= kDeferMinK, the row heads and their distances, flat
//              scans (sm_scan_flat), longer scans deferred.
constexpr int kVarFirst = 0;
constexpr int kVarLane = 1;
constexpr int kVarDefer = 3;
// LDS bytes of M for a variant
template <int V>
constexpr int var_ms_bytes() {
    return V == kVarDefer ? kMaxK * kRowPrefix : kMaxK * kRowStride;
}

// Finishes a block's deferred scans (Ms holds row heads of kRowPrefix
// entries, rows the whole rows in device memory), in three phases:
//   1. wave w takes queue entries w, w + NW, ..., each with sm_finish_wave
//      over the row past its head (the row entries of the first step of
//      kDeferBatch entries are loaded together), and writes the choice and
//      whether it is certified back into the entry; evaluations go to ev of
//      lane 0;
//   2. one thread per certified entry computes its float64 distance;
//   3. the other entries are decided by resolve_wave, one wave each.
// For each finished point rec(idx, key, count, best, float64 distance) is
// called by one thread (stores and LDS atomics only).  All threads call it,
// after a barrier that follows the last push to the queue.
constexpr uint32_t kDeferUnsure = 1u << 16;  // entry flag after phase 1

template <int NT, typename Rec>
__device__ __forceinline__ void finish_deferred(int K, int mode, const float4 *cen,
                                                const double4 *cen64, const uint8_t *Ms,
                                                const uint8_t *__restrict__ rows, DeferQueue *dq,
                                                uint32_t &ev, Rec &&rec) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t nd = dq->n < (uint32_t)kDeferCap ? dq->n : (uint32_t)kDeferCap;
    for (uint32_t q0 = wave; q0 < nd; q0 += NW * kDeferBatch) {
        int tf[kDeferBatch];
#pragma unroll
        for (int u = 0; u < kDeferBatch; ++u) {
            const uint32_t q = q0 + (uint32_t)(u * NW);
            tf[u] = 0;
            if (q < nd) {
                const uint32_t pjb = dq->pjb[q];
                const int jj = (int)(pjb >> 16) + lane;
                const size_t row = (size_t)((pjb >> 8) & 0xFFu) * kRowStride;
                if (jj < K - 1) tf[u] = rows[row + jj];
            }
        }
        // one entry per step; tf is rotated so that its first element is the
        // current entry's (the loop body is not unrolled)
#pragma unroll 1
        for (int u = 0; u < kDeferBatch; ++u) {
            const int t_first = tf[0];
#pragma unroll
            for (int v = 0; v + 1 < kDeferBatch; ++v) tf[v] = tf[v + 1];
            const uint32_t q = q0 + (uint32_t)(u * NW);
            if (q >= nd) break;  // wave-uniform
            const uint32_t pjb = dq->pjb[q];
            const int p = (int)((pjb >> 8) & 0xFFu);
            int best = (int)(pjb & 0xFFu);
            float bd = __uint_as_float(dq->bd[q]);
            float s2 = __uint_as_float(dq->s2[q]);
            float x, y, z;
            unpack_key(dq->key[q], x, y, z);
            const float4 cp = cen[p];
            const float prev = sq_dist(x, y, z, cp.x, cp.y, cp.z);
            const float thr = prev * kBreakScale;
            uint32_t sev = 0;
            float dj;
            const RowView rv{Ms + p * kRowPrefix, rows + (size_t)p * kRowStride, kRowPrefix};
            sm_finish_wave(x, y, z, p, K, cen, rv, thr, (int)(pjb >> 16), t_first, bd, best, s2,
                           dj, sev);
            // the results are the same in every lane
            const bool sure =
                mode == kModeExact || (mode == kModeCertify && certified(bd, s2, prev, dj));
            if (lane == 0) {
                ev += sev;
                dq->bd[q] = __float_as_uint(bd);
                dq->pjb[q] = (sure ? 0u : kDeferUnsure) | ((uint32_t)p << 8) | (uint32_t)best;
            }
        }
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < nd; q += NT) {
        const uint32_t pjb = dq->pjb[q];
        if (pjb & kDeferUnsure) continue;
        const int best = (int)(pjb & 0xFFu);
        const uint32_t k = dq->key[q];
        double d64;
        if (mode == kModeExact) {
            d64 = (double)__uint_as_float(dq->bd[q]);  // exact (integer centers)
        } else {
            const double4 cb = cen64[best];
            d64 = sq_dist64((double)((k >> 16) & 0xFFu), (double)((k >> 8) & 0xFFu),
                            (double)(k & 0xFFu), cb.x, cb.y, cb.z);
        }
        rec(dq->idx[q], k, dq->cnt[q], best, d64);
    }
    for (uint32_t c0 = (uint32_t)wave * 64u; c0 < nd; c0 += NW * 64u) {
        const uint32_t q = c0 + (uint32_t)lane;
        unsigned long long unsure = __ballot(q < nd && (dq->pjb[q] & kDeferUnsure) != 0u);
        while (unsure != 0ull) {  // wave-uniform
            const uint32_t qq = c0 + (uint32_t)__builtin_ctzll(unsure);
            unsure &= unsure - 1ull;
            const uint32_t k = dq->key[qq];
            const Choice64 c = resolve_wave(k, (int)((dq->pjb[qq] >> 8) & 0xFFu), K, cen64);
            if (lane == 0) rec(dq->idx[qq], k, dq->cnt[qq], c.best, c.d64);
        }
    }
}

// The number of evaluations the sort-means scan of x from p makes: 1 (the
// previous center) + the number of row entries before the first one at or
// past the threshold.  Row p is sorted by d(c_p, c_t)^2, so a binary search
// finds that position; the distances are recomputed with the scan's own
// expression.
__device__ __forceinline__ uint32_t sm_scan_evals(float x, float y, float z, int p, int K,
                                                  const float4 *cen, const uint8_t *Ms, int rs) {
    const float4 cp = cen[p];
    const float thr = sq_dist(x, y, z, cp.x, cp.y, cp.z) * kBreakScale;
    const uint8_t *row = Ms + p * rs;
    int lo = 0, hi = K - 1;  // first entry in [lo, hi] with d >= thr (hi: none)
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const float4 ct = cen[row[mid]];
        if (sq_dist(cp.x, cp.y, cp.z, ct.x, ct.y, ct.z) >= thr)
            hi = mid;
        else
            lo = mid + 1;
    }
    return 1u + (uint32_t)lo;
}

// Full search over all K centers with the same tie key; with TOP2 it also
// returns the second smallest distance (for certified()), otherwise s2_out
// is left alone (exact mode needs no certificate).
template <bool TOP2>
__device__ __forceinline__ int full_scan(float x, float y, float z, int p, int K,
                                         const float4 *cen, float &best_d, float &s2_out,
                                         uint32_t &ev) {
    const float4 cp = cen[p];
    const float prev = sq_dist(x, y, z, cp.x, cp.y, cp.z);
    float lo = TOP2 ? kNoSkip : prev, s2 = kNoSkip;
    int best = p;
    // Centers in ascending order, kScanBatch at a time (reads issued
    // together; cen has kMaxK entries, and those past K are not taken).
    // Under the tie rule (dist, k != p, k) a center replaces the best exactly
    // when it is strictly nearer: a later center that ties the best has a
    // higher index than it, or the best is still p, and both are kept; and
    // once the best has left p it is strictly nearer than p, so p (taken in
    // its turn, tying with the start) cannot tie it again.  With TOP2 the
    // scan starts empty instead, so that p is counted once among the two
    // smallest distances, and p wins a tie with the first center at the
    // smallest distance afterwards (its distance, recomputed by the same
    // expression, is prev).
    for (int t0 = 0; t0 < K; t0 += kScanBatch) {
        float d[kScanBatch];
#pragma unroll
        for (int e = 0; e < kScanBatch; ++e) {
            const float3 ct = *(const float3 *)(cen + t0 + e);
            d[e] = sq_dist(x, y, z, ct.x, ct.y, ct.z);
        }
#pragma unroll
        for (int e = 0; e < kScanBatch; ++e) {
            if (t0 + e < K) {
                if (TOP2) s2 = fminf(s2, fmaxf(d[e], lo));
                if (d[e] < lo) {
                    lo = d[e];
                    best = t0 + e;
                }
            }
        }
    }
    if (TOP2 && prev == lo) best = p;
    ev += (uint32_t)K;
    best_d = lo;
    if (TOP2) s2_out = s2;
    return best;
}

// Block sums of a double and a u64 in a fixed order: waves reduce with DPP,
// wave totals are added in wave order.  Results valid in thread 0.
template <int NT>
__device__ __forceinline__ void block_sum2(double &v, unsigned long long &e, double *dscr,
                                           unsigned long long *uscr) {
    v = wave_sum_f64(v);
    e = wave_sum_u64(e);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 63) {
        dscr[wave] = v;
        uscr[wave] = e;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        unsigned long long u = 0;
        for (int w = 0; w < NT / 64; ++w) {
            s += dscr[w];
            u += uscr[w];
        }
        v = s;
        e = u;
    }
}

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

}  // namespace wsm
