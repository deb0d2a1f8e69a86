// Device code of the weighted sort-means iterations (Alg. 2), shared by the
// per-image launches (iterate.hip) and the batched persistent form
// (batch.hip): the center update, the accumulation, the search over a
// block's points, and the bodies of the rows, search and final steps.  The
// step structure is described in iterate.hip.
#pragma once

#include <type_traits>

#include "sm_block.h"

namespace wsm {

struct IterArgs {
    StateView sv;
    Points pts;
    int k;
    int grid;          // blocks of the step kernel (partials per step)
    double eps;
    int64_t n_pixels;  // sum of the weights
};

// Center totals: packed as two u64 (sum cR | sum cG << 32, sum cB | sum c << 32)
// when 255 * n_pixels < 2^32, else four u64; center c's words are
// c * NW .. c * NW + NW - 1 (NW = 2 or 4) of each of the kTotCopies copies
// of a slot.  The center is the float64 quotient of the exact sums (their
// correctly rounded mean); an empty cluster keeps its center.
template <bool PACKED>
constexpr int tot_words() { return PACKED ? 2 : 4; }

// Words w < k * NW of the copies of slot T, summed into tot[w] (LDS), one
// word per thread with the loads of all copies issued together.  Packed
// words add field by field: no field of a total reaches 2^32, so no carry
// crosses a field.
template <int NT, bool PACKED>
__device__ __forceinline__ void gather_totals(const unsigned long long *T, int k,
                                              unsigned long long *tot) {
    for (int w = threadIdx.x; w < k * tot_words<PACKED>(); w += NT) {
        unsigned long long v[kTotCopies];
#pragma unroll
        for (int q = 0; q < kTotCopies; ++q) v[q] = T[q * kTotCopy + w];
        unsigned long long t = 0ull;
#pragma unroll
        for (int q = 0; q < kTotCopies; ++q) t += v[q];
        tot[w] = t;
    }
}

// Zeroes the words of the copies of slot T that k centers use.
template <int NT, bool PACKED>
__device__ __forceinline__ void clear_totals(unsigned long long *T, int k) {
#pragma unroll
    for (int q = 0; q < kTotCopies; ++q)
        for (int w = threadIdx.x; w < k * tot_words<PACKED>(); w += NT) T[q * kTotCopy + w] = 0ull;
}

template <bool PACKED>
__device__ __forceinline__ double4 totals_to_center(const unsigned long long *tot, int c,
                                                    double4 prev) {
    constexpr int NW = tot_words<PACKED>();
    unsigned long long sr, sg, sb, w;
    if (PACKED) {
        const unsigned long long a = tot[c * NW], b = tot[c * NW + 1];
        sr = a & 0xFFFFFFFFull;
        sg = a >> 32;
        sb = b & 0xFFFFFFFFull;
        w = b >> 32;
    } else {
        sr = tot[c * NW];
        sg = tot[c * NW + 1];
        sb = tot[c * NW + 2];
        w = tot[c * NW + 3];
    }
    if (w == 0ull) return prev;  // empty cluster keeps its center
    const double dw = (double)w;
    return make_double4((double)sr / dw, (double)sg / dw, (double)sb / dw, 0.0);
}

// Update phase (see the file comment).  Returns the record after the update,
// identical in every block, with the mode (kMode*) of the new centers.  The
// new centers are in the LDS array cen after the call, and in float64 in
// cen64 if it is not null.
template <int NT, bool PACKED>
__device__ Record update_phase(const IterArgs &a, int i, float4 *cen, double4 *cen64,
                               bool writer, double *dscr, unsigned long long *uscr,
                               unsigned long long *tot) {
    constexpr int kPer = kMaxK / NT > 0 ? kMaxK / NT : 1;
    const int tid = threadIdx.x;
    const Record rin = a.sv.hdr->rec[i & 1];
    const double4 *pal_in = a.sv.pal64 + (size_t)(i & 1) * kMaxK;
    float4 *pal_out = a.sv.pal + (size_t)((i + 1) & 1) * kMaxK;
    double4 *pal64_out = a.sv.pal64 + (size_t)((i + 1) & 1) * kMaxK;
    const int prv = (i + 2) % 3;  // totals slot of step i-1
    const unsigned long long *T = a.sv.totals + (size_t)prv * kTotSlot;
    // Issue every load first; which values are used is decided afterwards.
    const bool update = (i != 0) && !rin.converged;
    double4 cv[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int c = tid + r * NT;
        cv[r] = c < a.k ? pal_in[c] : make_double4(0.0, 0.0, 0.0, 0.0);
    }
    // Lane l of the first wave sums partials l, l + 64, l + 128, ... in that
    // order; the loads of eight of them are issued together.
    double s = 0.0;
    unsigned long long e = 0;
    if (tid < 64) {
        const double *sp = a.sv.sse_part + (size_t)((i + 1) & 1) * kMaxGrid;
        const unsigned long long *ep = a.sv.eval_part + (size_t)((i + 1) & 1) * kMaxGrid;
        for (int g0 = 0; g0 < a.grid; g0 += 64 * 8) {
            double v[8];
            unsigned long long w[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int g = g0 + u * 64 + tid;
                v[u] = g < a.grid ? sp[g] : 0.0;
                w[u] = g < a.grid ? ep[g] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                s += v[u];
                e += w[u];
            }
        }
    }
    gather_totals<NT, PACKED>(T, a.k, tot);
    __syncthreads();
    int flags = 0;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int c = tid + r * NT;
        if (c < a.k) {
            if (update) cv[r] = totals_to_center<PACKED>(tot, c, cv[r]);
            cen[c] = make_float4((float)cv[r].x, (float)cv[r].y, (float)cv[r].z, 0.0f);
            if (cen64) cen64[c] = cv[r];
            flags |= center_flags(cv[r]);
        }
    }
    Record r = rin;
    if (update) {
        // Weighted SSE of step i-1 from the per-block partials, reduced by
        // the first wave in a fixed order (identical in every block).
        if (tid < 64) {
            s = wave_sum_f64(s);
            e = wave_sum_u64(e);
            if (tid == 63) {
                dscr[0] = s;
                uscr[0] = e;
            }
        }
        __syncthreads();
        const double sse = dscr[0] / (double)a.n_pixels;
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
    // a barrier that also votes on the mode of the new centers: updated
    // centers are means of colors, so only a center kept from the initial
    // palette can lie outside [0, 256) (the flag set at init)
    const int nonint = __syncthreads_or(flags & kFlagNonInt);
    r.mode = a.sv.hdr->wild ? kModeResolve : nonint ? kModeCertify : kModeExact;
    if (writer) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int c = tid + q * NT;
            if (c < a.k) {
                pal_out[c] = cen[c];
                pal64_out[c] = cv[q];
            }
        }
        if (tid == 0) a.sv.hdr->rec[(i + 1) & 1] = r;
    }
    return r;
}

// Point of a state: packed key and weight.
__device__ __forceinline__ void load_point(const Points &P, int64_t idx, uint32_t &key,
                                           uint32_t &cnt) {
    if (P.is_pixels) {
        const uint8_t *px = P.rgb + idx * 3;
        key = ((uint32_t)px[0] << 16) | ((uint32_t)px[1] << 8) | (uint32_t)px[2];
        cnt = 1u;
    } else {
        key = P.colors[idx];
        cnt = P.counts[idx];
    }
}

// Add one point's weighted color to the block's LDS sums.  All lanes of the
// wave must call it; runs of equal centers are pre-summed first.
template <bool PACKED>
__device__ __forceinline__ void accumulate(unsigned long long *acc, int best, bool valid,
                                           uint32_t key, uint32_t cnt) {
    const unsigned long long c = valid ? (unsigned long long)cnt : 0ull;
    const unsigned long long r = (key >> 16) & 0xFFu, g = (key >> 8) & 0xFFu, b = key & 0xFFu;
    unsigned long long v0, v1, v2 = 0, v3 = 0;
    if (PACKED) {
        v0 = c * r | ((c * g) << 32);
        v1 = c * b | (c << 32);
    } else {
        v0 = c * r;
        v1 = c * g;
        v2 = c * b;
        v3 = c;
    }
    const int k = valid ? best : -1;
    const int head = run_head(k);
    wave_seg_sum2(head, v0, v1);
    if (!PACKED) wave_seg_sum2(head, v2, v3);
    if (run_tail(k, valid)) {
        if (PACKED) {
            atomicAdd(&acc[best * 2 + 0], v0);
            atomicAdd(&acc[best * 2 + 1], v1);
        } else {
            atomicAdd(&acc[best * 4 + 0], v0);
            atomicAdd(&acc[best * 4 + 1], v1);
            atomicAdd(&acc[best * 4 + 2], v2);
            atomicAdd(&acc[best * 4 + 3], v3);
        }
    }
}

// Points of (virtual) block vb of a step's a.grid blocks: the 64-point
// chunks vb, vb + grid, vb + 2 grid, ... of the (key-ordered) table, one
// chunk per wave and slot, so that every block samples the whole color range
// and the blocks get similar work.
__device__ __forceinline__ int64_t block_slots(const IterArgs &a, int vb) {
    const int64_t chunks = (a.pts.n + 63) / 64;
    const int64_t b = vb;
    return chunks > b ? (chunks - b + a.grid - 1) / a.grid : 0;
}

__device__ __forceinline__ int64_t slot_point(const IterArgs &a, int vb, int64_t slot) {
    return ((int64_t)vb + slot * a.grid) * 64 + (threadIdx.x & 63);
}

__device__ __forceinline__ void prefetch_points(const IterArgs &a, int vb, uint32_t (&key)[kCpt],
                                                uint32_t (&cnt)[kCpt], int (&pm)[kCpt]) {
    const int64_t ns = block_slots(a, vb);
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < kCpt; ++r) {
        const int64_t slot = r * (kSearchThreads / 64) + wave;
        const int64_t idx = slot_point(a, vb, slot);
        key[r] = 0u;
        cnt[r] = 0u;
        pm[r] = 0;
        if (slot < ns && idx < a.pts.n) {
            load_point(a.pts, idx, key[r], cnt[r]);
            pm[r] = a.sv.m[idx];
        }
    }
}

// Deferred sort-means scans (search kernel for K >= kDeferMinK): a point
// whose scan goes past the row head that sm_scan_flat covers goes to an LDS
// queue (DeferQueue; while it has room, otherwise its lane carries on alone)
// and is finished after the block's passes by a whole wave
// (finish_deferred), so that the rare long scans do not hold their wave.
// The first step of a call, when every point starts from center 0 and most
// scans are long, runs its own kernel (the full search), so the queue can
// stay short.

// End of a search block: finishes the deferred scans (DEFER), adds the
// block's sums into totals slot i % 3 and writes its SSE and evaluation
// partials.  All threads call it.
template <bool PACKED, bool DEFER>
__device__ void finish_block(const IterArgs &a, int i, int vb, int mode, const float4 *cen,
                             const double4 *cen64, const uint8_t *Ms, unsigned long long *acc,
                             double *dscr, unsigned long long *uscr, DeferQueue *dq, double sse,
                             uint32_t ev) {
    constexpr int NT = kSearchThreads;
    constexpr int NACC = PACKED ? 2 : 4;
    const int tid = threadIdx.x;
    if (DEFER) {
        __syncthreads();
        finish_deferred<NT>(a.k, mode, cen, cen64, Ms, a.sv.rows, dq, ev,
                            [&](uint32_t idx, uint32_t k, uint32_t c, int best, double d64) {
            sse += (double)c * d64;
            a.sv.m[idx] = (uint8_t)best;
            const unsigned long long cc = c;
            const unsigned long long rr = (k >> 16) & 0xFFu, gg = (k >> 8) & 0xFFu, bb = k & 0xFFu;
            if (PACKED) {
                atomicAdd(&acc[best * 2 + 0], cc * rr | ((cc * gg) << 32));
                atomicAdd(&acc[best * 2 + 1], cc * bb | (cc << 32));
            } else {
                atomicAdd(&acc[best * 4 + 0], cc * rr);
                atomicAdd(&acc[best * 4 + 1], cc * gg);
                atomicAdd(&acc[best * 4 + 2], cc * bb);
                atomicAdd(&acc[best * 4 + 3], cc);
            }
        });
    }
    __syncthreads();
    // this block's copy of the totals slot (see kTotCopies)
    unsigned long long *T =
        a.sv.totals + (size_t)(i % 3) * kTotSlot + (blockIdx.x % kTotCopies) * kTotCopy;
    for (int c = tid; c < a.k * NACC; c += NT) {
        const unsigned long long v = acc[c];
        if (v != 0ull) atomicAdd(&T[c], v);
    }
    unsigned long long e = ev;
    block_sum2<NT>(sse, e, dscr, uscr);
    if (tid == 0) {
        a.sv.sse_part[(size_t)(i & 1) * kMaxGrid + vb] = sse;
        a.sv.eval_part[(size_t)(i & 1) * kMaxGrid + vb] = e;
    }
}

// Search and accumulation over a block's points (block_slots): a first
// pass of kCpt 64-color slots per wave, whose points are already in
// key/cnt/pm, then slots taken one at a time from the block's counter.  Sort-means over the LDS copy Ms of M, or full
// search for the comparator (Ms unused); every choice is then made final in
// float64 by decide64 (mode: of the centers cen, whose float64 values are
// cen64), and the SSE is summed from float64 distances.  Adds the block's
// sums into totals slot i % 3 and writes its SSE and evaluation partials.

template <bool PACKED, bool FULL, bool DEFER, bool TAB = false>
__device__ void search_chunk(const IterArgs &a, int i, int vb, int mode, const float4 *cen,
                             const double4 *cen64, const uint8_t *Ms, unsigned long long *acc,
                             double *dscr, unsigned long long *uscr, DeferQueue *dq,
                             uint32_t *next, uint32_t (&key)[kCpt], uint32_t (&cnt)[kCpt],
                             int (&pm)[kCpt], bool first = false, const float *Dd = nullptr,
                             FlatScratch *fs = nullptr, const float4 *Tb = nullptr, int ts = 0) {
    constexpr int NT = kSearchThreads;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int rs = lds_rows_stride<DEFER>(a.k);
    const int64_t ns = block_slots(a, vb);
    double sse = 0.0;
    uint32_t ev = 0;
    // The wave's next slot past the first pass, taken from the block's
    // counter, and its point (loaded one round ahead).
    int64_t dslot = 0;
    uint32_t kd = 0u, cd = 0u;
    int pd = 0;
    auto take = [&]() {
        uint32_t t = 0u;
        if ((tid & 63) == 0) t = atomicAdd(next, 1u);
        dslot = kCpt * NW + (int64_t)__builtin_amdgcn_readfirstlane(t);
        const int64_t idx = slot_point(a, vb, dslot);
        kd = 0u;
        cd = 0u;
        pd = 0;
        if (dslot < ns && idx < a.pts.n) {
            load_point(a.pts, idx, kd, cd);
            pd = a.sv.m[idx];
        }
    };
    // One round per loop step: first the first pass's kCpt slots (r NW +
    // wave, whose points came with key/cnt/pm and are rotated so that the
    // round's point is element 0), then slots taken one at a time from the
    // block's counter, so that waves whose points scan long take fewer of
    // them.  The loop body is not unrolled.
#pragma unroll 1
    for (int r = 0;; ++r) {
        uint32_t kr, cr;
        int pr;
        int64_t slot;
        if (r < kCpt) {
            kr = key[0];
            cr = cnt[0];
            pr = pm[0];
#pragma unroll
            for (int v = 0; v + 1 < kCpt; ++v) {
                key[v] = key[v + 1];
                cnt[v] = cnt[v + 1];
                pm[v] = pm[v + 1];
            }
            slot = (int64_t)r * NW + wave;
            if (r == kCpt - 1 && slot < ns) take();
        } else {
            kr = kd;
            cr = cd;
            pr = pd;
            slot = dslot;
            if (slot < ns) take();
        }
        if (slot >= ns) break;  // wave-uniform; the slots a wave visits ascend
        {
            const int64_t idx = slot_point(a, vb, slot);
            const bool valid = slot < ns && idx < a.pts.n;
            float x, y, z;
            unpack_key(kr, x, y, z);
            float bd = 0.f, s2 = kNoSkip, prev = 0.f, dj = kNoSkip;
            int best = 0;
            bool done = true;
            if (FULL || first) {
                // the full search; or in the first step (every point starts
                // from center 0, whose whole row is scanned) the full search
                // gives the same center, and the scan's evaluation count
                // comes from a binary search of row p
                if (valid) {
                    uint32_t fev = 0;
                    if (mode == kModeExact)
                        best = full_scan<false>(x, y, z, pr, a.k, cen, bd, s2, fev);
                    else
                        best = full_scan<true>(x, y, z, pr, a.k, cen, bd, s2, fev);
                    ev += FULL ? fev : sm_scan_evals(x, y, z, pr, a.k, cen, Ms, rs);
                }
            } else if (TAB) {
                if (valid)
                    best = sm_scan_tab(x, y, z, pr, a.k, cen, Ms, rs, Tb, ts, bd, prev, s2, dj,
                                       ev);
            } else if (!DEFER) {
                if (valid) best = sm_scan(x, y, z, pr, a.k, cen, Ms, rs, bd, prev, s2, dj, ev);
            } else {
                // the wave's scans over the row heads together; a scan that
                // goes past the head is deferred (or, with the queue full,
                // carried on by its lane)
                float thr;
                bool more;
                sm_scan_flat(valid, kr, pr, a.k, cen, Ms, Dd, fs[wave], thr, prev, bd, s2,
                             dj, best, ev, more);
                if (more) {
                    const uint32_t q = atomicAdd(&dq->n, 1u);
                    if (q < (uint32_t)kDeferCap) {
                        dq->idx[q] = (uint32_t)idx;
                        dq->key[q] = kr;
                        dq->cnt[q] = cr;
                        dq->bd[q] = __float_as_uint(bd);
                        dq->s2[q] = __float_as_uint(s2);
                        dq->pjb[q] = ((uint32_t)kRowPrefix << 16) | ((uint32_t)pr << 8) |
                                     (uint32_t)best;
                        done = false;
                    } else {
                        const RowView rv{Ms + pr * rs, a.sv.rows + (size_t)pr * kRowStride,
                                         kRowPrefix};
                        int j = kRowPrefix;
                        dj = kNoSkip;
                        sm_scan_range(x, y, z, pr, a.k, cen, rv, thr, j, a.k, bd, best, s2, dj,
                                      ev);
                    }
                }
            }
            const bool fin = valid && done;
            const double d64 = decide64(fin, kr, pr, a.k, mode, cen64, best, bd, s2, prev,
                                        dj);
            if (fin) {
                a.sv.m[idx] = (uint8_t)best;
                sse += (double)cr * d64;
            }
            accumulate<PACKED>(acc, best, fin, kr, cr);
        }
    }
    finish_block<PACKED, DEFER>(a, i, vb, mode, cen, cen64, Ms, acc, dscr, uscr, dq, sse, ev);
}


// LDS of the step bodies below, as structs so that a kernel that runs
// several of them (the batched form) can overlay them.
struct RowsLds {
    float4 cen[kMaxK];
    unsigned long long tot[kMaxK * 4];
    __align__(16) unsigned long long keys[kMaxK];
    uint32_t rank[kMaxK];
    double dscr[kSortThreads / 64];
    unsigned long long uscr[kSortThreads / 64];
};

template <int V>
struct SearchLds {
    static constexpr bool kDefer = V == kVarDefer;
    float4 cen[kMaxK];
    double4 cen64[kMaxK];
    unsigned long long acc[kMaxK * 4];
    // rows of M: the first kRowPrefix entries when scans defer, else whole
    __align__(16) uint8_t Ms[var_ms_bytes<V>()];
    // kVarDefer: the distances of the row heads, and the flat scans' scratch
    __align__(16) float Dd[kDefer ? kMaxK * kRowDist : 4];
    FlatScratch fs[kDefer ? kSearchThreads / 64 : 1];
    typename std::conditional<kDefer, DeferQueue, NoQueue>::type dq;
    double dscr[kSearchThreads / 64];
    unsigned long long uscr[kSearchThreads / 64];
    uint32_t next;  // the block's slot counter past the first pass
};

template <int V>
__device__ __forceinline__ DeferQueue *queue_of(SearchLds<V> &L) {
    if constexpr (V == kVarDefer)
        return &L.dq;
    else
        return nullptr;
}

template <int NT>
struct FinalLds {
    float4 cen[kMaxK];
    unsigned long long tot[kMaxK * 4];
    double4 cen64[kMaxK];
    double dscr[NT / 64];
    unsigned long long uscr[NT / 64];
};

// Sort-means step i, rows part (kSortThreads threads): the update of step
// i-1 (see the file comment of iterate.hip), then rows p0 .. p1-1 of M for
// the new centers.  The part with p0 == 0 publishes the update and clears
// the totals slot step i accumulates into.
template <bool PACKED>
__device__ void rows_body(const IterArgs &a, int i, int p0, int p1, RowsLds &L) {
    const Record rec =
        update_phase<kSortThreads, PACKED>(a, i, L.cen, nullptr, p0 == 0, L.dscr, L.uscr, L.tot);
    if (rec.converged) return;
    if (p0 == 0) {
        clear_totals<kSortThreads, PACKED>(a.sv.totals + (size_t)(i % 3) * kTotSlot, a.k);
    }
    for (int p = p0; p < p1; ++p)
        sort_row<kSortThreads>(L.cen, a.k, p, L.keys, L.rank, a.sv.rows + (size_t)p * kRowStride,
                               a.sv.rowd + (size_t)p * kRowDist);
}

// Sort-means step i, search part (kSearchThreads threads), block vb of
// a.grid: the centers and M copied into LDS, then the block's points.
template <bool PACKED, int V>
__device__ void search_body(const IterArgs &a, int i, int vb, SearchLds<V> &L) {
    constexpr int NT = kSearchThreads;
    constexpr int NACC = PACKED ? 2 : 4;
    constexpr bool DEFER = V == kVarDefer, FIRST = V == kVarFirst;
    const int tid = threadIdx.x;
    uint32_t key[kCpt], cnt[kCpt];
    int pm[kCpt];
    prefetch_points(a, vb, key, cnt, pm);
    // This step's centers and rows are fetched before the record is read, so
    // the loads overlap (they are only used if the loop has not stopped).
    const float4 *pal = a.sv.pal + (size_t)((i + 1) & 1) * kMaxK;
    const float4 pc = tid < a.k ? pal[tid] : make_float4(0.f, 0.f, 0.f, 0.f);
    const double4 *pal64 = a.sv.pal64 + (size_t)((i + 1) & 1) * kMaxK;
    const double4 pc64 = tid < a.k ? pal64[tid] : make_double4(0.0, 0.0, 0.0, 0.0);
    RowRegs<NT> R;
    fetch_rows<NT, DEFER>(a.sv.rows, a.k, R);
    constexpr int kDdRegs = DEFER ? kMaxK * kRowDist / 4 / NT : 1;  // 16-byte pieces per thread
    static_assert(!DEFER || kMaxK * kRowDist / 4 == kDdRegs * NT, "distance copy");
    uint4 dreg[kDdRegs];
    if (DEFER) {
#pragma unroll
        for (int u = 0; u < kDdRegs; ++u) {
            const int q = tid + u * NT;
            dreg[u] = q < a.k * (kRowDist / 4) ? ((const uint4 *)a.sv.rowd)[q]
                                               : make_uint4(0u, 0u, 0u, 0u);
        }
    }
    const Record rec = a.sv.hdr->rec[(i + 1) & 1];
    if (rec.converged) return;
    if (tid < a.k) {
        L.cen[tid] = pc;
        L.cen64[tid] = pc64;
    }
    store_rows<NT, DEFER>(R, a.k, L.Ms);
    if (DEFER) {
#pragma unroll
        for (int u = 0; u < kDdRegs; ++u) {
            const int q = tid + u * NT;
            if (q < a.k * (kRowDist / 4)) ((uint4 *)L.Dd)[q] = dreg[u];
        }
    }
    for (int c = tid; c < a.k * NACC; c += NT) L.acc[c] = 0ull;
    if (tid == 0) L.next = 0u;
    if constexpr (DEFER) {
        if (tid == 0) L.dq.n = 0u;
    }
    __syncthreads();

    // The launch for a call's first step (FIRST) checks whether the state has
    // completed no step yet, i.e. every membership is still 0 (state init).
    const bool first = FIRST && rec.iters == 0;
    search_chunk<PACKED, false, DEFER>(a, i, vb, rec.mode, L.cen, L.cen64, L.Ms, L.acc, L.dscr,
                                       L.uscr, queue_of(L), &L.next, key, cnt, pm, first, L.Dd,
                                       L.fs);
}


// The update of step i-1 alone (one block of NT threads): published, with
// the record, for step i; unless the stopping rule has fired, the totals
// slot step i accumulates into is cleared.  Returns the record.
template <int NT, bool PACKED>
__device__ Record update_body(const IterArgs &a, int i, FinalLds<NT> &L) {
    const Record r = update_phase<NT, PACKED>(a, i, L.cen, L.cen64, true, L.dscr, L.uscr, L.tot);
    if (!r.converged) {
        clear_totals<NT, PACKED>(a.sv.totals + (size_t)(i % 3) * kTotSlot, a.k);
    }
    __syncthreads();
    __threadfence();
    return r;
}

// Rows p0 .. p1-1 of M for the centers published for step i (kSortThreads
// threads).
__device__ void sort_body(const IterArgs &a, int i, int p0, int p1, RowsLds &L) {
    const float4 *pal = a.sv.pal + (size_t)((i + 1) & 1) * kMaxK;
    for (int c = threadIdx.x; c < a.k; c += kSortThreads) L.cen[c] = pal[c];
    for (int p = p0; p < p1; ++p)  // sort_row starts with a barrier
        sort_row<kSortThreads>(L.cen, a.k, p, L.keys, L.rank, a.sv.rows + (size_t)p * kRowStride,
                               a.sv.rowd + (size_t)p * kRowDist);
}

// Final update after the last step of a call (one block of NT threads).
// Publishes the palette and record to slot 0 and clears totals[0] for the
// next call.
template <int NT, bool PACKED>
__device__ void final_body(const IterArgs &a, int i, FinalLds<NT> &L) {
    const int tid = threadIdx.x;
    const Record r = update_phase<NT, PACKED>(a, i, L.cen, L.cen64, true, L.dscr, L.uscr, L.tot);
    __syncthreads();
    for (int c = tid; c < a.k; c += NT) {
        a.sv.pal[c] = L.cen[c];
        a.sv.pal64[c] = L.cen64[c];
    }
    unsigned long long *T0 = a.sv.totals;
    for (int c = tid; c < (int)kTotSlot; c += NT) T0[c] = 0ull;
    if (tid == 0) {
        a.sv.hdr->rec[0] = r;
        a.sv.hdr->info[0] = r.iters;
        a.sv.hdr->info[1] = r.converged;
        a.sv.hdr->info[2] = r.err;
        a.sv.hdr->info[3] = 0;
    }
}


}  // namespace wsm
