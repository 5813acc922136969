// Optional per-kernel timing with hipEvents (diagnostics API of hawkes.h).
#include <hip/hip_runtime.h>
#include <mutex>
#include <vector>
#include "hk_internal.h"

namespace hk {

struct TimedLaunch {
    int id;
    hipEvent_t a, b;
};

static std::mutex g_mu;
static uint32_t g_mask = 0;   // kernels whose launches are timed
static std::vector<TimedLaunch> g_pending;
static double g_ms[HAWKES_TIMING_KERNELS];
static int64_t g_cnt[HAWKES_TIMING_KERNELS];

static void drain_locked() {
    for (auto& L : g_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(L.b) == hipSuccess && hipEventElapsedTime(&ms, L.a, L.b) == hipSuccess) {
            g_ms[L.id] += ms;
            g_cnt[L.id] += 1;
        }
        (void)hipEventDestroy(L.a);
        (void)hipEventDestroy(L.b);
    }
    g_pending.clear();
}

bool timing_on() { return g_mask != 0; }

void* timing_begin(int id, hipStream_t st) {
    if (id < 0 || id >= HAWKES_TIMING_KERNELS || !((g_mask >> id) & 1u)) return nullptr;
    TimedLaunch* L = new TimedLaunch{id, nullptr, nullptr};
    if (hipEventCreate(&L->a) != hipSuccess || hipEventCreate(&L->b) != hipSuccess ||
        hipEventRecord(L->a, st) != hipSuccess) {
        delete L;
        return nullptr;
    }
    return L;
}

void timing_end(void* h, hipStream_t st) {
    if (!h) return;
    TimedLaunch* L = (TimedLaunch*)h;
    if (hipEventRecord(L->b, st) == hipSuccess) {
        std::lock_guard<std::mutex> g(g_mu);
        g_pending.push_back(*L);
    }
    delete L;
}

}  // namespace hk

extern "C" {

hawkes_status hawkes_timing_enable(int on) {
    std::lock_guard<std::mutex> g(hk::g_mu);
    hk::g_mask = on < 0 ? 0xffffffffu : (uint32_t)on;
    return HAWKES_OK;
}

hawkes_status hawkes_timing_reset(void) {
    std::lock_guard<std::mutex> g(hk::g_mu);
    hk::drain_locked();
    for (int i = 0; i < HAWKES_TIMING_KERNELS; ++i) { hk::g_ms[i] = 0.0; hk::g_cnt[i] = 0; }
    return HAWKES_OK;
}

hawkes_status hawkes_timing_read(int kernel_id, double* total_ms, int64_t* launches) {
    if (kernel_id < 0 || kernel_id >= HAWKES_TIMING_KERNELS || !total_ms || !launches) return HAWKES_EINVAL;
    std::lock_guard<std::mutex> g(hk::g_mu);
    hk::drain_locked();
    *total_ms = hk::g_ms[kernel_id];
    *launches = hk::g_cnt[kernel_id];
    return HAWKES_OK;
}

}  // extern "C"
