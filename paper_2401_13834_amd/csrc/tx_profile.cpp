// Per-kernel launch timing with hipEvents recorded on the launch stream.
#include <atomic>

#include "tx_internal.h"

namespace {

struct Slot {
    hipEvent_t start = nullptr, end = nullptr;
    int kernel = -1;
    bool used = false;
};

std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<Slot> g_slots;

}  // namespace

namespace tx {

int prof_begin(int kernel, hipStream_t stream) {
    if (!g_on.load(std::memory_order_relaxed)) return -1;
    std::lock_guard<std::mutex> lock(g_mu);
    int idx = -1;
    for (size_t i = 0; i < g_slots.size(); ++i)
        if (!g_slots[i].used) {
            idx = static_cast<int>(i);
            break;
        }
    if (idx < 0) {
        Slot s;
        if (hipEventCreate(&s.start) != hipSuccess) return -1;
        if (hipEventCreate(&s.end) != hipSuccess) {
            (void)hipEventDestroy(s.start);
            return -1;
        }
        g_slots.push_back(s);
        idx = static_cast<int>(g_slots.size() - 1);
    }
    Slot& s = g_slots[idx];
    if (hipEventRecord(s.start, stream) != hipSuccess) return -1;
    s.kernel = kernel;
    s.used = true;
    return idx;
}

void prof_end(int slot, hipStream_t stream) {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lock(g_mu);
    if (hipEventRecord(g_slots[slot].end, stream) != hipSuccess) g_slots[slot].used = false;
}

}  // namespace tx

extern "C" {

tx_status tx_profile_enable(int32_t on) {
    g_on.store(on ? 1 : 0);
    return TX_OK;
}

tx_status tx_profile_collect(int32_t kernel, double* total_ms, int64_t* launches) {
    if (kernel < 0 || kernel >= TX_KERNEL_COUNT || !total_ms || !launches) return TX_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    double sum = 0.0;
    int64_t n = 0;
    for (Slot& s : g_slots) {
        if (!s.used || s.kernel != kernel) continue;
        if (hipEventSynchronize(s.end) != hipSuccess) return TX_EDEVICE;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, s.start, s.end) != hipSuccess) return TX_EDEVICE;
        sum += ms;
        ++n;
        s.used = false;
    }
    *total_ms = sum;
    *launches = n;
    return TX_OK;
}

}  // extern "C"
