// Batched persistent form of the weighted sort-means iterations on gfx950:
// many images, each with its own table of unique colors, K and iteration
// budget, iterated by one launch of persistent blocks that take work items
// from a device queue.
//
// An image's steps are those of the per-image launches (iterate.hip), cut
// into work items:
//   start item (image):     the first step's centers published
//                           (update_body);
//   rows item (image, r):   rows r * rpi .. (r + 1) * rpi - 1 of M for the
//                           step's centers (sort_body);
//   search item (image, v): virtual block v of the image's search grid
//                           (search_body).
// The block that completes the last item of a phase goes on with the image:
// after the rows, it enqueues the search items; after the search, it applies
// the update once (update_body) -- or the final update (final_body) when the
// iteration budget is spent or the Sec. 3.2 criterion has fired, ending the
// image -- and enqueues the next step's rows items.  Images interleave
// freely, so small images and the short phases of one image fill the GPU
// together.
//
// Queue protocol (device memory of the caller's workspace): a block claims
// the next slot with an atomic on `head` and waits until the slot's ready
// word holds this run's number; a producer reserves slots with an atomic on
// `tail`, writes the items, fences, and stores the run number into their
// ready words.  Slots are claimed in order, so a waiting block only ever
// waits for items that running blocks will produce; when no image is left
// every waiting block leaves.  A bounded wait sets an error bit instead of
// spinning forever.  The run number grows by one per launch, so ready words
// of earlier runs never match.
#include <cstring>
#include <new>
#include <vector>

#include "iter_device.h"

int wsm_internal_check_problem(const wsm_problem *prob);

namespace wsm {

constexpr int kBatchMaxImages = 128;
constexpr uint32_t kItemRows = 0u;
constexpr uint32_t kItemSearch = 1u;
constexpr uint32_t kItemStart = 2u;
constexpr uint32_t kNoItem = ~0u;
// longest wait for one slot, in ticks of the constant 100 MHz realtime
// counter (2 s; a whole batch takes milliseconds)
constexpr unsigned long long kWaitTicks = 200000000ull;
constexpr int32_t kErrSpin = 1;             // a block gave up waiting for an item
constexpr int32_t kErrOverflow = 2;         // the queue ran out of slots

struct BatchImage {
    IterArgs a;
    int32_t max_iters;
    int32_t rows_per_item;
    int32_t rows_items;   // ceil(k / rows_per_item)
    int32_t pad;
};

struct BatchCtl {
    uint32_t head;        // next slot to claim
    uint32_t tail;        // next slot to reserve
    uint32_t run;         // number of the current launch
    uint32_t cap;         // slots
    int32_t remaining;    // images not finished
    int32_t err;          // kErr* bits
    int32_t n_images;
    int32_t pad;
};

struct ImgCtl {
    uint32_t step;        // call-relative step of the current phase
    uint32_t done;        // completed items of the current phase
    uint32_t pad[2];
};

__host__ __device__ constexpr uint32_t make_item(uint32_t image, uint32_t kind, uint32_t index) {
    return (image << 25) | (kind << 23) | index;
}

union BatchLds {
    SearchLds<kVarDefer> d;
    SearchLds<kVarLane> l;
    SearchLds<kVarFirst> n;
    RowsLds r;
    FinalLds<kSearchThreads> f;
};

// Resets the queue for a launch: the next run number, one start item per
// image.  One block.
__global__ __launch_bounds__(256) void batch_reset_kernel(const BatchImage *__restrict__ img,
                                                          BatchCtl *ctl, ImgCtl *ictl,
                                                          uint32_t *items, uint32_t *ready) {
    __shared__ uint32_t s_run;
    const int n = ctl->n_images;
    if (threadIdx.x == 0) {
        s_run = ctl->run + 1u;
        ctl->run = s_run;
        ctl->head = 0u;
        ctl->remaining = n;
        ctl->err = 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        items[i] = make_item((uint32_t)i, kItemStart, 0u);
        ready[i] = s_run;
        ictl[i].step = 0u;
        ictl[i].done = 0u;
    }
    if (threadIdx.x == 0) ctl->tail = (uint32_t)n;
}

// Appends n_new items (image, kind, 0..n_new-1) to the queue.  All threads
// call it.
__device__ void enqueue(BatchCtl *ctl, uint32_t *items, uint32_t *ready, uint32_t run,
                        uint32_t image, uint32_t kind, uint32_t n_new, uint32_t *s_base) {
    __syncthreads();
    if (threadIdx.x == 0) *s_base = atomicAdd(&ctl->tail, n_new);
    __syncthreads();
    const uint32_t base = *s_base;
    if (base + n_new > ctl->cap) {
        if (threadIdx.x == 0) {
            atomicOr(&ctl->err, kErrOverflow);
            __threadfence();
            atomicSub(&ctl->remaining, 1);  // the image cannot go on
        }
        return;
    }
    for (uint32_t j = threadIdx.x; j < n_new; j += blockDim.x)
        items[base + j] = make_item(image, kind, j);
    __syncthreads();
    // one release fence (the first wave's), after which that wave publishes
    // the ready words: the block's item stores come before it
    if (threadIdx.x < 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        for (uint32_t j = threadIdx.x; j < n_new; j += 64)
            __hip_atomic_store(&ready[base + j], run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ __launch_bounds__(kSearchThreads) void batch_kernel(const BatchImage *__restrict__ img,
                                                               BatchCtl *ctl, ImgCtl *ictl,
                                                               uint32_t *items, uint32_t *ready) {
    __shared__ BatchLds L;
    __shared__ uint32_t s_item, s_base;
    __shared__ int s_last;
    const int tid = threadIdx.x;
    const uint32_t run = ctl->run;
    const uint32_t cap = ctl->cap;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            uint32_t item = kNoItem;
            const uint32_t slot = atomicAdd(&ctl->head, 1u);
            const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
            // relaxed polls; one acquire fence once the slot is ready (an
            // acquire at every poll would invalidate the L2 each time)
            for (;;) {
                if (slot < cap && __hip_atomic_load(&ready[slot], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT) == run) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    item = items[slot];
                    break;
                }
                if (__hip_atomic_load(&ctl->remaining, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT) <= 0)
                    break;
                if (__builtin_amdgcn_s_memrealtime() - t0 > kWaitTicks) {
                    atomicOr(&ctl->err, kErrSpin);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            s_item = item;
        }
        __syncthreads();
        // the item is the same for the whole block: scalar registers
        const uint32_t item = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_item);
        if (item == kNoItem) return;
        const uint32_t im = item >> 25, kind = (item >> 23) & 3u, idx = item & 0x7FFFFFu;
        const BatchImage &B = img[im];
        const IterArgs a = B.a;
        const int step = __builtin_amdgcn_readfirstlane((int)ictl[im].step);
        if (kind == kItemStart) {
            // the first step's centers (a state that had already converged
            // is final at once)
            const Record rec = update_body<kSearchThreads, true>(a, 0, L.f);
            if (rec.converged) {
                final_body<kSearchThreads, true>(a, 1, L.f);
                __syncthreads();
                if (tid == 0) {
                    __threadfence();
                    atomicSub(&ctl->remaining, 1);
                }
            } else {
                enqueue(ctl, items, ready, run, im, kItemRows, (uint32_t)B.rows_items, &s_base);
            }
            continue;
        }
        if (kind == kItemRows) {
            const int p0 = (int)idx * B.rows_per_item;
            const int p1 = p0 + B.rows_per_item < a.k ? p0 + B.rows_per_item : a.k;
            sort_body(a, step, p0, p1, L.r);
        } else if (step == 0) {
            search_body<true, kVarFirst>(a, step, (int)idx, L.n);
        } else if (a.k >= kDeferMinK) {
            search_body<true, kVarDefer>(a, step, (int)idx, L.d);
        } else {
            search_body<true, kVarLane>(a, step, (int)idx, L.l);
        }
        // completion of the item; the last one of the phase goes on
        __syncthreads();
        if (tid == 0) {
            const uint32_t total = kind == kItemRows ? (uint32_t)B.rows_items : (uint32_t)a.grid;  // start items return above
            // release the block's results, count the item; the last one
            // acquires everyone else's
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t old = atomicAdd(&ictl[im].done, 1u);
            s_last = (old + 1u == total) ? 1 : 0;
            if (s_last) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                // ready for the next phase's items, which are published later
                // (after the release fence in enqueue)
                __hip_atomic_store(&ictl[im].done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
        if (!s_last) continue;
        bool finished = false;
        if (kind == kItemRows) {
            enqueue(ctl, items, ready, run, im, kItemSearch, (uint32_t)a.grid, &s_base);
        } else if (step + 1 >= B.max_iters) {
            final_body<kSearchThreads, true>(a, step + 1, L.f);
            finished = true;
        } else {
            const Record rec = update_body<kSearchThreads, true>(a, step + 1, L.f);
            if (rec.converged) {
                final_body<kSearchThreads, true>(a, step + 2, L.f);
                finished = true;
            } else {
                if (tid == 0) {
                    ictl[im].step = (uint32_t)(step + 1);
                    __threadfence();
                }
                enqueue(ctl, items, ready, run, im, kItemRows, (uint32_t)B.rows_items, &s_base);
            }
        }
        if (finished) {
            __syncthreads();
            if (tid == 0) {
                __threadfence();
                atomicSub(&ctl->remaining, 1);
            }
        }
    }
}

// Clears the ready words once, when a plan is made.
__global__ void batch_clear_kernel(uint32_t *ready, uint32_t cap, BatchCtl *ctl, int n_images) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < cap; j += stride) ready[j] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->head = ctl->tail = 0u;
        ctl->run = 0u;
        ctl->cap = cap;
        ctl->remaining = 0;
        ctl->err = 0;
        ctl->n_images = n_images;
        ctl->pad = 0;
    }
}

struct BatchLayout {
    size_t off_ctl, off_img, off_ictl, off_items, off_ready, bytes;
    uint32_t cap;
};

}  // namespace wsm

using namespace wsm;

// ---------------------------------------------------------------------------
// Host side.

struct wsm_batch {
    uint32_t magic;
    int n_images;
    int grid;                 // persistent blocks
    hipGraphExec_t exec;      // reset + persistent launch
    BatchCtl *ctl;            // device
    BatchImage *img;          // device
    ImgCtl *ictl;
    uint32_t *items, *ready;
};

constexpr uint32_t kBatchMagic = 0x574D4242u;

static int batch_layout(int n_images, const wsm_problem *probs, const int32_t *max_iters,
                        const int32_t *grid, const int32_t *rows_per_item, BatchLayout &L) {
    if (!probs || !max_iters || n_images < 1 || n_images > kBatchMaxImages) return WSM_EINVAL;
    uint64_t items = 0;
    for (int i = 0; i < n_images; ++i) {
        const wsm_problem &p = probs[i];
        if (wsm_internal_check_problem(&p) != WSM_OK) return WSM_EINVAL;
        if (p.points != WSM_POINTS_COLORS) return WSM_EINVAL;
        if ((unsigned long long)p.n_pixels * 255ull >= (1ull << 32)) return WSM_EINVAL;
        if (max_iters[i] < 1 || max_iters[i] > kHistory) return WSM_EINVAL;
        const int g = grid && grid[i] > 0 ? grid[i] : p.grid;
        if (g < 1 || g > kMaxGrid) return WSM_EINVAL;
        const int rpi = rows_per_item && rows_per_item[i] > 0 ? rows_per_item[i] : 1;
        if (rpi > kMaxK) return WSM_EINVAL;
        const int ri = (p.k + rpi - 1) / rpi;
        items += 1 + (uint64_t)max_iters[i] * (uint64_t)(ri + g);
    }
    // every persistent block claims one slot past the last item when it leaves
    items += 4096;
    if (items > 0x7FFFFFFFull) return WSM_EINVAL;
    L.cap = (uint32_t)items;
    L.off_ctl = 0;
    L.off_img = align_up(sizeof(BatchCtl), 256);
    L.off_ictl = align_up(L.off_img + sizeof(BatchImage) * (size_t)n_images, 256);
    L.off_items = align_up(L.off_ictl + sizeof(ImgCtl) * (size_t)n_images, 256);
    L.off_ready = align_up(L.off_items + 4ull * L.cap, 256);
    L.bytes = align_up(L.off_ready + 4ull * L.cap, 256);
    return WSM_OK;
}

extern "C" int wsm_batch_workspace_bytes(int n_images, const wsm_problem *probs,
                                         const int32_t *max_iters, const int32_t *grid,
                                         const int32_t *rows_per_item, size_t *bytes) {
    if (!bytes) return WSM_EINVAL;
    BatchLayout L;
    const int rc = batch_layout(n_images, probs, max_iters, grid, rows_per_item, L);
    if (rc != WSM_OK) return rc;
    *bytes = L.bytes;
    return WSM_OK;
}

extern "C" int wsm_batch_create(int n_images, const wsm_problem *probs, const int32_t *max_iters,
                                const double *eps, const int32_t *grid,
                                const int32_t *rows_per_item, void *workspace,
                                size_t workspace_bytes, wsm_batch **batch) {
    if (!batch || !eps || !workspace) return WSM_EINVAL;
    *batch = nullptr;
    BatchLayout L;
    int rc = batch_layout(n_images, probs, max_iters, grid, rows_per_item, L);
    if (rc != WSM_OK) return rc;
    if (workspace_bytes < L.bytes) return WSM_ENOSPC;
    if (((uintptr_t)workspace & 255u) != 0u) return WSM_EINVAL;
    std::vector<BatchImage> host((size_t)n_images);
    for (int i = 0; i < n_images; ++i) {
        if (!(eps[i] >= 0.0) || eps[i] > 1e300) return WSM_EINVAL;
        const wsm_problem &p = probs[i];
        BatchImage &b = host[(size_t)i];
        std::memset(&b, 0, sizeof(b));
        b.a.sv = make_view(p.state);
        b.a.pts.colors = p.colors;
        b.a.pts.counts = p.counts;
        b.a.pts.rgb = p.rgb;
        b.a.pts.n = p.n_points;
        b.a.pts.is_pixels = 0;
        b.a.k = p.k;
        b.a.grid = grid && grid[i] > 0 ? grid[i] : p.grid;
        b.a.eps = eps[i];
        b.a.n_pixels = p.n_pixels;
        b.max_iters = max_iters[i];
        b.rows_per_item = rows_per_item && rows_per_item[i] > 0 ? rows_per_item[i] : 1;
        b.rows_items = (p.k + b.rows_per_item - 1) / b.rows_per_item;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return WSM_EHIP;
    char *ws = (char *)workspace;
    wsm_batch *h = new (std::nothrow) wsm_batch;
    if (!h) return WSM_EHIP;
    h->magic = kBatchMagic;
    h->n_images = n_images;
    h->grid = cus > 0 ? cus : 1;  // one 1024-thread block per CU (its LDS use allows no more)
    h->ctl = (BatchCtl *)(ws + L.off_ctl);
    h->img = (BatchImage *)(ws + L.off_img);
    h->ictl = (ImgCtl *)(ws + L.off_ictl);
    h->items = (uint32_t *)(ws + L.off_items);
    h->ready = (uint32_t *)(ws + L.off_ready);
    h->exec = nullptr;
    // set-up, synchronous: descriptors and cleared ready words
    (void)hipGetLastError();
    rc = WSM_EHIP;
    hipStream_t cs = nullptr;
    if (hipMemcpy(h->img, host.data(), sizeof(BatchImage) * host.size(), hipMemcpyHostToDevice) ==
            hipSuccess &&
        hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess) {
        batch_clear_kernel<<<dim3(256), dim3(256), 0, cs>>>(h->ready, L.cap, h->ctl, n_images);
        hipGraph_t g = nullptr;
        if (hipGetLastError() == hipSuccess && hipStreamSynchronize(cs) == hipSuccess &&
            hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            batch_reset_kernel<<<dim3(1), dim3(256), 0, cs>>>(h->img, h->ctl, h->ictl, h->items,
                                                              h->ready);
            batch_kernel<<<dim3((unsigned)h->grid), dim3(kSearchThreads), 0, cs>>>(
                h->img, h->ctl, h->ictl, h->items, h->ready);
            const hipError_t launched = hipGetLastError();
            const hipError_t end = hipStreamEndCapture(cs, &g);
            if (launched == hipSuccess && end == hipSuccess && g &&
                hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0) == hipSuccess)
                rc = WSM_OK;
        }
        if (g) (void)hipGraphDestroy(g);
    }
    if (cs) (void)hipStreamDestroy(cs);
    (void)hipGetLastError();
    if (rc != WSM_OK) {
        delete h;
        return rc;
    }
    *batch = h;
    return WSM_OK;
}

extern "C" int wsm_batch_launch(wsm_batch *batch, hipStream_t stream) {
    if (!batch || batch->magic != kBatchMagic) return WSM_EINVAL;
    return hipGraphLaunch(batch->exec, stream) == hipSuccess ? WSM_OK : WSM_EHIP;
}

extern "C" int wsm_batch_error(const wsm_batch *batch, const int32_t **err) {
    if (!batch || batch->magic != kBatchMagic || !err) return WSM_EINVAL;
    *err = &batch->ctl->err;
    return WSM_OK;
}

extern "C" int wsm_batch_destroy(wsm_batch *batch) {
    if (!batch) return WSM_OK;
    if (batch->magic != kBatchMagic) return WSM_EINVAL;
    const hipError_t e = hipGraphExecDestroy(batch->exec);
    batch->magic = 0u;
    delete batch;
    return e == hipSuccess ? WSM_OK : WSM_EHIP;
}
