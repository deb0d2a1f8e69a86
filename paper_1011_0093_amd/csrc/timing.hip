// Measurement hook of the C ABI: while attached, every launch of one chosen
// kernel is made with hipExtLaunchKernelGGL and a pair of HIP events that
// the runtime records when the kernel starts and ends, on the stream it is
// launched on, so a caller can time that kernel's launches inside a larger
// sequence without a profiler.  Not used on the normal path.
#include <atomic>
#include <mutex>
#include <vector>

#include "wsm_internal.h"

namespace {

struct TimingState {
    int which = 0;
    int capacity = 0;
    int count = 0;
    std::vector<hipEvent_t> begin, end;
};

TimingState g_timing;
std::mutex g_timing_mu;          // guards g_timing
std::atomic<int> g_timed_kind{0};  // g_timing.which, read without the lock by every launch

}  // namespace

namespace wsm {

bool timing_claim(int kind, hipEvent_t *begin, hipEvent_t *end) {
    if (g_timed_kind.load(std::memory_order_acquire) != kind) return false;
    std::lock_guard<std::mutex> lock(g_timing_mu);
    if (g_timing.which != kind || g_timing.count >= g_timing.capacity) return false;
    *begin = g_timing.begin[g_timing.count];
    *end = g_timing.end[g_timing.count];
    ++g_timing.count;
    return true;
}

}  // namespace wsm

extern "C" int wsm_timing_attach(int which, int capacity) {
    if (which < WSM_KERNEL_REDUCE_PARTITION || which > WSM_KERNEL_FULL_STEP || capacity < 1 ||
        capacity > (1 << 20))
        return WSM_EINVAL;
    std::lock_guard<std::mutex> lock(g_timing_mu);
    if (g_timing.which != 0) return WSM_EINVAL;
    g_timing.begin.assign(capacity, nullptr);
    g_timing.end.assign(capacity, nullptr);
    for (int i = 0; i < capacity; ++i) {
        if (hipEventCreate(&g_timing.begin[i]) != hipSuccess ||
            hipEventCreate(&g_timing.end[i]) != hipSuccess) {
            for (int j = 0; j <= i; ++j) {
                if (g_timing.begin[j]) (void)hipEventDestroy(g_timing.begin[j]);
                if (g_timing.end[j]) (void)hipEventDestroy(g_timing.end[j]);
            }
            g_timing.begin.clear();
            g_timing.end.clear();
            return WSM_EHIP;
        }
    }
    g_timing.capacity = capacity;
    g_timing.count = 0;
    g_timing.which = which;
    g_timed_kind.store(which, std::memory_order_release);
    return WSM_OK;
}

extern "C" int wsm_timing_read(float *ms, int capacity, int *count) {
    if (!count || (capacity > 0 && !ms)) return WSM_EINVAL;
    std::lock_guard<std::mutex> lock(g_timing_mu);
    if (g_timing.which == 0) return WSM_EINVAL;
    const int n = g_timing.count < capacity ? g_timing.count : capacity;
    for (int i = 0; i < n; ++i) {
        if (hipEventSynchronize(g_timing.end[i]) != hipSuccess) return WSM_EHIP;
        if (hipEventElapsedTime(&ms[i], g_timing.begin[i], g_timing.end[i]) != hipSuccess)
            return WSM_EHIP;
    }
    *count = g_timing.count;
    return WSM_OK;
}

extern "C" int wsm_timing_detach(void) {
    std::lock_guard<std::mutex> lock(g_timing_mu);
    if (g_timing.which == 0) return WSM_OK;
    g_timed_kind.store(0, std::memory_order_release);
    for (size_t i = 0; i < g_timing.begin.size(); ++i) {
        (void)hipEventSynchronize(g_timing.end[i]);
        (void)hipEventDestroy(g_timing.begin[i]);
        (void)hipEventDestroy(g_timing.end[i]);
    }
    g_timing = TimingState();
    return WSM_OK;
}
