// Iterations of the weighted sort-means loop (Alg. 2) on gfx950: two
// launches per iteration (one for the full-search comparator).
//
// Step i, rows launch (one block per center p):
//   1. every block applies the center update of step i-1 (Alg. 2, last
//      loop: c_k = sum w x / sum w, from exact integer sums of
//      count * channel), reduces the SSE partials of step i-1 in a fixed
//      order and evaluates the Sec. 3.2 stopping rule -- redundantly, so all
//      blocks agree without a grid-wide barrier; block 0 publishes the
//      palette and the record;
//   2. block p sorts row p of the neighbour matrix M for the new centers
//      (Sec. 2: the inter-center distances with every row sorted).
// Step i, search launch (one block per chunk of points):
//   3. sort-means from each point's previous center over an LDS copy of M
//      (for K >= kDeferMinK a wave's scans over the row heads are spread
//      over its lanes, and the rare longer ones finished by whole waves);
//   4. sums count * (R, G, B, 1) per center: runs of equal centers within a
//      wave are pre-summed with a segmented scan, then added into LDS, and
//      each block flushes its non-zero sums with 64-bit device atomics (the
//      second level of the reduction); the block's SSE and evaluation count
//      go to per-block partials.
// The full-search comparator does 1, 3 (full search) and 4 in one launch.
// The sums are exact integers, so the result does not depend on the order
// of the additions and the pruned search, the full search and k-means on the
// raw pixels produce bit-identical centers.
//
// Records and palettes are double-buffered by step parity and the totals
// triple-buffered, so no launch reads what another block of the same launch
// writes.  A single-block kernel applies the final update after the last
// step and copies the result to the public slot 0.
#include <new>

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
// when 255 * n_pixels < 2^32, else four u64.  The center is the float64
// quotient of the exact sums (their correctly rounded mean); an empty
// cluster keeps its center.
template <bool PACKED>
__device__ __forceinline__ void totals_to_center(const unsigned long long *T, int c,
                                                 double4 prev, double4 &out) {
    unsigned long long sr, sg, sb, w;
    if (PACKED) {
        const unsigned long long a = T[c * 4 + 0], b = T[c * 4 + 1];
        sr = a & 0xFFFFFFFFull;
        sg = a >> 32;
        sb = b & 0xFFFFFFFFull;
        w = b >> 32;
    } else {
        sr = T[c * 4 + 0];
        sg = T[c * 4 + 1];
        sb = T[c * 4 + 2];
        w = T[c * 4 + 3];
    }
    if (w != 0ull) {
        const double dw = (double)w;
        out = make_double4((double)sr / dw, (double)sg / dw, (double)sb / dw, 0.0);
    } else {
        out = prev;  // empty cluster keeps its center
    }
}

// Update phase (see the file comment).  Returns the record after the update,
// identical in every block, with the mode (kMode*) of the new centers.  The
// new centers are in the LDS array cen after the call, and in float64 in
// cen64 if it is not null.
template <int NT, bool PACKED>
__device__ Record update_phase(const IterArgs &a, int i, float4 *cen, double4 *cen64,
                               bool writer, double *dscr, unsigned long long *uscr) {
    constexpr int kPer = kMaxK / NT > 0 ? kMaxK / NT : 1;
    const int tid = threadIdx.x;
    const Record rin = a.sv.hdr->rec[i & 1];
    const double4 *pal_in = a.sv.pal64 + (size_t)(i & 1) * kMaxK;
    float4 *pal_out = a.sv.pal + (size_t)((i + 1) & 1) * kMaxK;
    double4 *pal64_out = a.sv.pal64 + (size_t)((i + 1) & 1) * kMaxK;
    const int prv = (i + 2) % 3;  // totals slot of step i-1
    const unsigned long long *T = a.sv.totals + (size_t)prv * kMaxK * 4;
    // Issue every load first; which values are used is decided afterwards.
    const bool update = (i != 0) && !rin.converged;
    double4 cv[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int c = tid + r * NT;
        cv[r] = make_double4(0.0, 0.0, 0.0, 0.0);
        if (c < a.k) {
            const double4 old = pal_in[c];
            double4 upd;
            totals_to_center<PACKED>(T, c, old, upd);
            cv[r] = update ? upd : old;
        }
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
    int flags = 0;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int c = tid + r * NT;
        if (c < a.k) {
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

// Points of a block: the 64-point chunks b, b + grid, b + 2 grid, ... of the
// (key-ordered) table, one chunk per wave and slot, so that every block
// samples the whole color range and the blocks get similar work.
__device__ __forceinline__ int64_t block_slots(const IterArgs &a) {
    const int64_t chunks = (a.pts.n + 63) / 64;
    const int64_t b = blockIdx.x;
    return chunks > b ? (chunks - b + a.grid - 1) / a.grid : 0;
}

__device__ __forceinline__ int64_t slot_point(const IterArgs &a, int64_t slot) {
    return ((int64_t)blockIdx.x + slot * a.grid) * 64 + (threadIdx.x & 63);
}

__device__ __forceinline__ void prefetch_points(const IterArgs &a, uint32_t (&key)[kCpt],
                                                uint32_t (&cnt)[kCpt], int (&pm)[kCpt]) {
    const int64_t ns = block_slots(a);
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < kCpt; ++r) {
        const int64_t slot = r * (kSearchThreads / 64) + wave;
        const int64_t idx = slot_point(a, slot);
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
__device__ void finish_block(const IterArgs &a, int i, int mode, const float4 *cen,
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
    unsigned long long *T = a.sv.totals + (size_t)(i % 3) * kMaxK * 4;
    for (int c = tid; c < a.k * NACC; c += NT) {
        const unsigned long long v = acc[c];
        if (v != 0ull) atomicAdd(&T[(c / NACC) * 4 + (c % NACC)], v);
    }
    unsigned long long e = ev;
    block_sum2<NT>(sse, e, dscr, uscr);
    if (tid == 0) {
        a.sv.sse_part[(size_t)(i & 1) * kMaxGrid + blockIdx.x] = sse;
        a.sv.eval_part[(size_t)(i & 1) * kMaxGrid + blockIdx.x] = e;
    }
}

// Search and accumulation over a block's points (block_slots), in passes of
// kPass (kCpt points per thread); the first pass's points are already in
// key/cnt/pm.  Sort-means over the LDS copy Ms of M, or full
// search for the comparator (Ms unused); every choice is then made final in
// float64 by decide64 (mode: of the centers cen, whose float64 values are
// cen64), and the SSE is summed from float64 distances.  Adds the block's
// sums into totals slot i % 3 and writes its SSE and evaluation partials.

template <bool PACKED, bool FULL, bool DEFER>
__device__ void search_chunk(const IterArgs &a, int i, int mode, const float4 *cen,
                             const double4 *cen64, const uint8_t *Ms, unsigned long long *acc,
                             double *dscr, unsigned long long *uscr, DeferQueue *dq,
                             uint32_t (&key)[kCpt], uint32_t (&cnt)[kCpt], int (&pm)[kCpt],
                             bool first = false, const float *Dd = nullptr,
                             FlatScratch *fs = nullptr) {
    constexpr int NT = kSearchThreads;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int rs = lds_rows_stride<DEFER>(a.k);
    const int64_t ns = block_slots(a);
    double sse = 0.0;
    uint32_t ev = 0;
    for (int64_t s0 = 0; s0 < ns; s0 += kCpt * NW) {
        if (s0 != 0) {
#pragma unroll
            for (int r = 0; r < kCpt; ++r) {
                const int64_t slot = s0 + r * NW + wave;
                const int64_t idx = slot_point(a, slot);
                if (slot < ns && idx < a.pts.n) {
                    load_point(a.pts, idx, key[r], cnt[r]);
                    pm[r] = a.sv.m[idx];
                }
            }
        }
        // one round per step, the points rotated so that the round's point
        // is element 0 (the loop body is not unrolled)
#pragma unroll 1
        for (int r = 0; r < kCpt; ++r) {
            const uint32_t kr = key[0], cr = cnt[0];
            const int pr = pm[0];
#pragma unroll
            for (int v = 0; v + 1 < kCpt; ++v) {
                key[v] = key[v + 1];
                cnt[v] = cnt[v + 1];
                pm[v] = pm[v + 1];
            }
            if (s0 + r * NW >= ns) break;  // block-uniform
            const int64_t slot = s0 + r * NW + wave;
            const int64_t idx = slot_point(a, slot);
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
    finish_block<PACKED, DEFER>(a, i, mode, cen, cen64, Ms, acc, dscr, uscr, dq, sse, ev);
}

// Sort-means step i, first launch: the update of step i-1 in every block
// (see the file comment), then block p sorts row p of M for the new
// centers.  Block 0 clears the totals slot step i accumulates into.
template <bool PACKED>
__global__ __launch_bounds__(kSortThreads) void rows_kernel(IterArgs a, int i) {
    __shared__ float4 cen[kMaxK];
    __shared__ __align__(16) unsigned long long keys[kMaxK];
    __shared__ uint32_t rank[kMaxK];
    __shared__ double dscr[kSortThreads / 64];
    __shared__ unsigned long long uscr[kSortThreads / 64];
    const int p = blockIdx.x;
    const Record rec = update_phase<kSortThreads, PACKED>(a, i, cen, nullptr, p == 0, dscr, uscr);
    if (rec.converged) return;
    if (p == 0) {
        unsigned long long *T = a.sv.totals + (size_t)(i % 3) * kMaxK * 4;
        for (int c = threadIdx.x; c < kMaxK * 4; c += kSortThreads) T[c] = 0ull;
    }
    sort_row<kSortThreads>(cen, a.k, p, keys, rank, a.sv.rows + (size_t)p * kRowStride,
                           a.sv.rowd + (size_t)p * kRowDist);
}

// Sort-means step i, second launch: every block copies the centers and M
// into LDS and searches its chunk.
template <bool PACKED, bool DEFER, bool FIRST>
__global__ __launch_bounds__(kSearchThreads) void search_kernel(IterArgs a, int i) {
    __shared__ float4 cen[kMaxK];
    __shared__ double4 cen64[kMaxK];
    __shared__ unsigned long long acc[kMaxK * 4];
    // rows of M: the first kRowPrefix entries when scans defer, else whole
    __shared__ __align__(16) uint8_t Ms[kMaxK * (DEFER ? kRowPrefix : kRowStride)];
    // with DEFER: the distances of those entries, and the flat scans' scratch
    __shared__ __align__(16) float Dd[DEFER ? kMaxK * kRowDist : 4];
    __shared__ FlatScratch fs[DEFER ? kSearchThreads / 64 : 1];
    __shared__ DeferQueue dq;
    __shared__ double dscr[kSearchThreads / 64];
    __shared__ unsigned long long uscr[kSearchThreads / 64];
    constexpr int NT = kSearchThreads;
    constexpr int NACC = PACKED ? 2 : 4;
    const int tid = threadIdx.x;
    uint32_t key[kCpt], cnt[kCpt];
    int pm[kCpt];
    prefetch_points(a, key, cnt, pm);
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
        cen[tid] = pc;
        cen64[tid] = pc64;
    }
    store_rows<NT, DEFER>(R, a.k, Ms);
    if (DEFER) {
#pragma unroll
        for (int u = 0; u < kDdRegs; ++u) {
            const int q = tid + u * NT;
            if (q < a.k * (kRowDist / 4)) ((uint4 *)Dd)[q] = dreg[u];
        }
    }
    for (int c = tid; c < a.k * NACC; c += NT) acc[c] = 0ull;
    if (tid == 0) dq.n = 0u;
    __syncthreads();
    // The launch for a call's first step (FIRST) checks whether the state has
    // completed no step yet, i.e. every membership is still 0 (state init).
    const bool first = FIRST && rec.iters == 0;
    search_chunk<PACKED, false, DEFER>(a, i, rec.mode, cen, cen64, Ms, acc, dscr, uscr, &dq, key,
                                       cnt, pm, first, Dd, fs);
}

// Rows of M for palette slot 0 of the state (the pixel map's palette).
__global__ __launch_bounds__(kSortThreads) void palette_rows_kernel(StateView sv, int K) {
    __shared__ float4 cen[kMaxK];
    __shared__ __align__(16) unsigned long long keys[kMaxK];
    __shared__ uint32_t rank[kMaxK];
    for (int c = threadIdx.x; c < K; c += kSortThreads) cen[c] = sv.pal[c];
    sort_row<kSortThreads>(cen, K, blockIdx.x, keys, rank, sv.rows + (size_t)blockIdx.x * kRowStride,
                           sv.rowd + (size_t)blockIdx.x * kRowDist);
}

// Sort-means step for K <= kFusedMaxK in one launch: every block applies
// the update as in the rows launch, sorts all K rows of M into LDS itself
// (thread (p, t) ranks center t in row p) and searches its points.  Totals
// slots follow the comparator's order: clear (i + 1) % 3, add into i % 3.
template <bool PACKED>
__global__ __launch_bounds__(kSearchThreads) void fused_step_kernel(IterArgs a, int i) {
    __shared__ float4 cen[kMaxK];
    __shared__ double4 cen64[kMaxK];
    __shared__ unsigned long long acc[kMaxK * 4];
    __shared__ __align__(16) unsigned long long keys[kFusedMaxK * kFusedMaxK];
    __shared__ __align__(16) uint8_t Ms[kFusedMaxK * kFusedMaxK];
    __shared__ double dscr[kSearchThreads / 64];
    __shared__ unsigned long long uscr[kSearchThreads / 64];
    constexpr int NT = kSearchThreads;
    constexpr int NACC = PACKED ? 2 : 4;
    static_assert(kFusedMaxK * kFusedMaxK <= NT, "one thread per row entry");
    const int tid = threadIdx.x;
    const int K = a.k;
    uint32_t key[kCpt], cnt[kCpt];
    int pm[kCpt];
    prefetch_points(a, key, cnt, pm);
    const Record rec = update_phase<NT, PACKED>(a, i, cen, cen64, blockIdx.x == 0, dscr, uscr);
    if (rec.converged) return;
    if (blockIdx.x == 0) {
        unsigned long long *Tn = a.sv.totals + (size_t)((i + 1) % 3) * kMaxK * 4;
        for (int c = tid; c < kMaxK * 4; c += NT) Tn[c] = 0ull;
    }
    for (int c = tid; c < K * NACC; c += NT) acc[c] = 0ull;
    const int p = tid / kFusedMaxK, t = tid % kFusedMaxK;
    const bool entry = p < K && t < K && t != p;
    unsigned long long kt = ~0ull;
    if (entry) {
        const float4 cp = cen[p], ct = cen[t];
        kt = ((unsigned long long)__float_as_uint(sq_dist(cp.x, cp.y, cp.z, ct.x, ct.y, ct.z))
              << 32) | (unsigned)t;
    }
    keys[tid] = kt;
    __syncthreads();
    if (entry) {
        const ulonglong2 *k2 = (const ulonglong2 *)(keys + p * kFusedMaxK);
        uint32_t r = 0;
#pragma unroll
        for (int u = 0; u < kFusedMaxK / 2; ++u) {
            const ulonglong2 v = k2[u];
            r += (uint32_t)(v.x < kt) + (uint32_t)(v.y < kt);
        }
        Ms[p * lds_row_stride(K) + r] = (uint8_t)t;
    }
    __syncthreads();
    search_chunk<PACKED, false, false>(a, i, rec.mode, cen, cen64, Ms, acc, dscr, uscr, nullptr,
                                       key, cnt, pm);
}

// Full-search comparator: one launch per step, the update applied
// redundantly by every block as in the sort-means step.
template <bool PACKED>
__global__ __launch_bounds__(kSearchThreads) void full_step_kernel(IterArgs a, int i) {
    __shared__ float4 cen[kMaxK];
    __shared__ double4 cen64[kMaxK];
    __shared__ unsigned long long acc[kMaxK * 4];
    __shared__ double dscr[kSearchThreads / 64];
    __shared__ unsigned long long uscr[kSearchThreads / 64];
    constexpr int NT = kSearchThreads;
    constexpr int NACC = PACKED ? 2 : 4;
    const int tid = threadIdx.x;
    uint32_t key[kCpt], cnt[kCpt];
    int pm[kCpt];
    prefetch_points(a, key, cnt, pm);
    const Record rec = update_phase<NT, PACKED>(a, i, cen, cen64, blockIdx.x == 0, dscr, uscr);
    if (rec.converged) return;
    if (blockIdx.x == 0) {
        unsigned long long *Tn = a.sv.totals + (size_t)((i + 1) % 3) * kMaxK * 4;
        for (int c = tid; c < kMaxK * 4; c += NT) Tn[c] = 0ull;
    }
    for (int c = tid; c < a.k * NACC; c += NT) acc[c] = 0ull;
    __syncthreads();
    search_chunk<PACKED, true, false>(a, i, rec.mode, cen, cen64, nullptr, acc, dscr, uscr,
                                      nullptr, key, cnt, pm);
}

// Final update after the last step of a call (one block).  Publishes the
// palette and record to slot 0 and clears totals[0] for the next call.
template <bool PACKED>
__global__ __launch_bounds__(kRowThreads) void final_kernel(IterArgs a, int i) {
    __shared__ float4 cen[kMaxK];
    __shared__ double4 cen64[kMaxK];
    __shared__ double dscr[4];
    __shared__ unsigned long long uscr[4];
    const int tid = threadIdx.x;
    const Record r = update_phase<kRowThreads, PACKED>(a, i, cen, cen64, true, dscr, uscr);
    __syncthreads();
    for (int c = tid; c < a.k; c += kRowThreads) {
        a.sv.pal[c] = cen[c];
        a.sv.pal64[c] = cen64[c];
    }
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
        int flags = 0;
        for (int c = 0; c < k; ++c)
            flags |= center_flags(make_double4((double)init_palette[3 * c],
                                               (double)init_palette[3 * c + 1],
                                               (double)init_palette[3 * c + 2], 0.0));
        h->wild = (flags & kFlagWild) ? 1 : 0;
        h->pad = 0;
        for (int j = 0; j < 3; ++j) h->reserved[j] = 0ull;
        Record z;
        z.iters = 0;
        z.converged = 0;
        z.err = 0;
        z.mode = kModeResolve;
        z.sse_last = 0.0;
        z.pad2 = 0.0;
        h->rec[0] = z;
        h->rec[1] = z;
        for (int j = 0; j < 4; ++j) h->info[j] = 0;
    }
    for (int64_t c = gt; c < 2 * kMaxK; c += stride) {
        const int64_t j = c % kMaxK;  // both slots hold the initial palette
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j < k) v = make_float4(init_palette[3 * j], init_palette[3 * j + 1],
                                   init_palette[3 * j + 2], 0.f);
        sv.pal[c] = v;
        sv.pal64[c] = make_double4((double)v.x, (double)v.y, (double)v.z, 0.0);
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
    // One block per CU, fewer for small tables (at least 256 points per
    // block), more when a block would otherwise need more than two passes.
    int64_t grid = cus;
    const int64_t by_size = (n_points + 255) / 256;
    if (by_size < grid) grid = by_size;
    const int64_t by_pass = (n_points + 2 * (int64_t)kPass - 1) / (2 * (int64_t)kPass);
    if (by_pass > grid) grid = by_pass;
    if (grid > kMaxGrid) grid = kMaxGrid;
    if (grid < 1) grid = 1;
    StateView sv = make_view(state);
    (void)hipGetLastError();
    init_state_kernel<<<dim3(256), dim3(256), 0, stream>>>(sv, k, points, (int)grid, n_points,
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
    prob->grid = (int)grid;
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
    if (prob->n_pixels < 1 || prob->n_pixels > (int64_t)0xFFFFFFFFll) return WSM_EINVAL;
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

int wsm_internal_check_problem(const wsm_problem *prob) { return check_problem(prob); }

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
    a.n_pixels = prob->n_pixels;
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

// Exact packing of the four sums into two 64-bit words needs 255 N < 2^32.
static bool packed_sums(const wsm_problem *prob) {
    return (unsigned long long)prob->n_pixels * 255ull < (1ull << 32);
}

template <bool PACKED>
static int launch_steps(const IterArgs &a, int max_iters, bool full, hipStream_t stream) {
    for (int i = 0; i < max_iters; ++i) {
        if (full) {
            WSM_LAUNCH(WSM_KERNEL_FULL_STEP, full_step_kernel<PACKED>, dim3(a.grid),
                       dim3(kSearchThreads), stream, a, i);
        } else if (a.k <= kFusedMaxK) {
            WSM_LAUNCH(WSM_KERNEL_SEARCH, fused_step_kernel<PACKED>, dim3(a.grid),
                       dim3(kSearchThreads), stream, a, i);
        } else {
            WSM_LAUNCH(WSM_KERNEL_ROWS, rows_kernel<PACKED>, dim3(a.k), dim3(kSortThreads), stream,
                       a, i);
            const auto search = i == 0 ? search_kernel<PACKED, false, true>
                                : a.k >= kDeferMinK ? search_kernel<PACKED, true, false>
                                                    : search_kernel<PACKED, false, false>;
            WSM_LAUNCH(WSM_KERNEL_SEARCH, search, dim3(a.grid), dim3(kSearchThreads), stream, a,
                       i);
        }
    }
    final_kernel<PACKED><<<dim3(1), dim3(kRowThreads), 0, stream>>>(a, max_iters);
    return hipGetLastError() == hipSuccess ? WSM_OK : WSM_EHIP;
}

// Rows of M for the state's published palette (used by the pixel map).
int wsm_internal_palette_rows(void *state, int k, hipStream_t stream) {
    palette_rows_kernel<<<dim3(k), dim3(kSortThreads), 0, stream>>>(make_view(state), k);
    return hipGetLastError() == hipSuccess ? WSM_OK : WSM_EHIP;
}

static int launch_direct(const IterArgs &a, int max_iters, bool full, bool packed,
                         hipStream_t stream) {
    return packed ? launch_steps<true>(a, max_iters, full, stream)
                  : launch_steps<false>(a, max_iters, full, stream);
}

static int iterate_impl(const wsm_problem *prob, int max_iters, double eps, bool full,
                        hipStream_t stream) {
    int rc = check_iter_args(prob, max_iters, eps);
    if (rc != WSM_OK) return rc;
    const IterArgs a = make_args(prob, eps);
    (void)hipGetLastError();
    return launch_direct(a, max_iters, full, packed_sums(prob), stream);
}

// ---------------------------------------------------------------------------
// A caller-owned HIP graph of one call's launch sequence.  The sequence
// depends only on the call's arguments, so it is recorded once (on a stream
// the create call makes and destroys) and replayed by every launch.
struct wsm_graph {
    uint32_t magic;
    hipGraphExec_t exec;
};

constexpr uint32_t kGraphMagic = 0x574D4752u;

extern "C" int wsm_iterate_graph_create(const wsm_problem *prob, int max_iters, double eps,
                                        int full, wsm_graph **graph) {
    if (!graph) return WSM_EINVAL;
    *graph = nullptr;
    int rc = check_iter_args(prob, max_iters, eps);
    if (rc != WSM_OK) return rc;
    const IterArgs a = make_args(prob, eps);
    (void)hipGetLastError();
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return WSM_EHIP;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    rc = WSM_EHIP;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        const int lrc = launch_direct(a, max_iters, full != 0, packed_sums(prob), cs);
        const hipError_t end = hipStreamEndCapture(cs, &g);
        if (lrc == WSM_OK && end == hipSuccess && g &&
            hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess)
            rc = WSM_OK;
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    (void)hipGetLastError();
    if (rc != WSM_OK) return rc;
    wsm_graph *h = new (std::nothrow) wsm_graph;
    if (!h) {
        (void)hipGraphExecDestroy(exec);
        return WSM_EHIP;
    }
    h->magic = kGraphMagic;
    h->exec = exec;
    *graph = h;
    return WSM_OK;
}

extern "C" int wsm_iterate_graph_launch(wsm_graph *graph, hipStream_t stream) {
    if (!graph || graph->magic != kGraphMagic) return WSM_EINVAL;
    return hipGraphLaunch(graph->exec, stream) == hipSuccess ? WSM_OK : WSM_EHIP;
}

extern "C" int wsm_iterate_graph_destroy(wsm_graph *graph) {
    if (!graph) return WSM_OK;
    if (graph->magic != kGraphMagic) return WSM_EINVAL;
    const hipError_t e = hipGraphExecDestroy(graph->exec);
    graph->magic = 0u;
    delete graph;
    return e == hipSuccess ? WSM_OK : WSM_EHIP;
}

extern "C" int wsm_iterate(const wsm_problem *prob, int max_iters, double eps,
                           hipStream_t stream) {
    return iterate_impl(prob, max_iters, eps, false, stream);
}

extern "C" int wsm_iterate_full(const wsm_problem *prob, int max_iters, double eps,
                                hipStream_t stream) {
    return iterate_impl(prob, max_iters, eps, true, stream);
}

extern "C" int wsm_state_views(const wsm_problem *prob, wsm_views *views) {
    if (!views) return WSM_EINVAL;
    int rc = check_problem(prob);
    if (rc != WSM_OK) return rc;
    const StateView sv = make_view(prob->state);
    views->palette = (const float *)sv.pal;
    views->palette64 = (const double *)sv.pal64;
    views->membership = sv.m;
    views->sse_history = sv.sse_hist;
    views->evals_history = (const int64_t *)sv.eval_hist;
    views->info = sv.hdr->info;
    return WSM_OK;
}

extern "C" int wsm_gather_palette(const uint32_t *colors, int64_t n_colors,
                                  const int32_t *indices, int k, float *palette,
                                  hipStream_t stream) {
    if (!colors || !indices || !palette || n_colors < 1 || k < 1 || k > kMaxK) return WSM_EINVAL;
    (void)hipGetLastError();
    gather_palette_kernel<<<dim3(1), dim3(kMaxK), 0, stream>>>(colors, n_colors, indices, k,
                                                               palette);
    return hipGetLastError() == hipSuccess ? WSM_OK : WSM_EHIP;
}
