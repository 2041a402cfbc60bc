// Tile autotuner: time every first-stage variant (and LDS size) with the
// second stage fixed, then every second-stage variant with the best first
// stage, on a scratch block of the plan's shape, and keep the fastest pair.
// Sums are exact integers, so every choice gives the same output.
#include <algorithm>
#include <vector>

#include "tx_internal.h"

namespace {

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

extern "C" tx_status tx_plan_autotune(tx_plan_t p, int64_t nt, int32_t effort, double* best_ms, hipStream_t stream) {
    if (!p || nt < 1 || nt > (int64_t(1) << 30) || effort < 0 || effort > 1) return TX_EINVAL;
    if (!p->on_device) return TX_ESTATE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TX_EDEVICE;
    if (dev != p->device) return TX_ESTATE;
    tx_status st = tx::retain_pool(dev);
    if (st != TX_OK) return st;

    std::vector<int> ldss = {0};
    // LDS sizes at the workgroups-per-CU steps of a 160 KB CU: 7, 6, 5, 4, 3.
    if (effort >= 1) ldss = {23392, 27296, 32768, 40960, 54608};
    std::vector<tx::Tiles> s1c, s2c;
    for (int v = 0; v < tx::stage1_variant_count(); ++v)
        for (int l : ldss) s1c.push_back(tx::Tiles{v, l, -1, 0});
    for (int v = 0; v < tx::stage2_variant_count(); ++v)
        for (int l : ldss) s2c.push_back(tx::Tiles{-1, 0, v, l});

    // Scratch sized for the largest geometry of any pair that can run: every
    // first-stage candidate with the default second stage, then the chosen
    // first stage (any of them) with every second-stage candidate.  The
    // first-stage series' pitch depends on both stages' tiles.
    int64_t ws_bytes = 0;
    for (const auto& c1 : s1c) {
        tx::DedispGeom g = tx::dedisp_geometry(p, nt, c1);
        if (g.ok) ws_bytes = std::max(ws_bytes, g.ws_bytes);
        for (const auto& c2 : s2c) {
            g = tx::dedisp_geometry(p, nt, tx::Tiles{c1.s1, c1.s1_lds, c2.s2, c2.s2_lds});
            if (g.ok) ws_bytes = std::max(ws_bytes, g.ws_bytes);
        }
    }
    const int64_t in_pitch = (nt + p->overlap + 255) / 256 * 256;
    const int64_t out_pitch = (nt + 1) / 2 * 2;
    void *in = nullptr, *out = nullptr, *ws = nullptr;
    hipError_t e = hipMallocAsync(&in, static_cast<size_t>(in_pitch) * p->nchan, stream);
    if (e == hipSuccess) e = hipMallocAsync(&out, static_cast<size_t>(out_pitch) * p->ndm * 4, stream);
    if (e == hipSuccess) e = hipMallocAsync(&ws, static_cast<size_t>(std::max<int64_t>(ws_bytes, 256)), stream);
    // The sums do not depend on the sample values; any bytes will do.
    if (e == hipSuccess) e = hipMemsetAsync(in, 0x5a, static_cast<size_t>(in_pitch) * p->nchan, stream);
    Timer tm;
    if (e == hipSuccess) e = hipEventCreate(&tm.a);
    if (e == hipSuccess) e = hipEventCreate(&tm.b);

    auto run = [&](const tx::Tiles& t, float* ms) -> hipError_t {
        const tx::DedispGeom g = tx::dedisp_geometry(p, nt, t);
        if (!g.ok || g.ws_bytes > ws_bytes) {       // the second never happens: sized above
            *ms = -1.0f;
            return hipSuccess;
        }
        auto once = [&]() {
            return tx::launch_dedisperse(p, g, static_cast<const uint8_t*>(in), in_pitch, nt,
                                         static_cast<int32_t*>(out), out_pitch, static_cast<uint16_t*>(ws), stream);
        };
        hipError_t r = once();                                   // warm-up
        if (r != hipSuccess) return r;
        r = hipEventRecord(tm.a, stream);
        if (r != hipSuccess) return r;
        r = once();
        if (r == hipSuccess) r = hipEventRecord(tm.b, stream);
        if (r == hipSuccess) r = hipEventSynchronize(tm.b);
        float one = 0.0f;
        if (r == hipSuccess) r = hipEventElapsedTime(&one, tm.a, tm.b);
        if (r != hipSuccess) return r;
        // Short runs: repeat so that one measurement covers about 2 ms.
        const int reps = std::min(50, std::max(1, static_cast<int>(2.0f / std::max(one, 1e-3f))));
        r = hipEventRecord(tm.a, stream);
        for (int k = 0; k < reps && r == hipSuccess; ++k) r = once();
        if (r == hipSuccess) r = hipEventRecord(tm.b, stream);
        if (r == hipSuccess) r = hipEventSynchronize(tm.b);
        float total = 0.0f;
        if (r == hipSuccess) r = hipEventElapsedTime(&total, tm.a, tm.b);
        *ms = std::min(one, total / static_cast<float>(reps));
        return r;
    };

    tx::Tiles best{-1, 0, -1, 0};
    float best_t = -1.0f;
    for (const auto& c : s1c) {
        if (e != hipSuccess) break;
        float ms = 0.0f;
        e = run(c, &ms);
        if (e == hipSuccess && ms >= 0.0f && (best_t < 0.0f || ms < best_t)) {
            best_t = ms;
            best.s1 = c.s1;
            best.s1_lds = c.s1_lds;
        }
    }
    for (const auto& c : s2c) {
        if (e != hipSuccess) break;
        tx::Tiles t = best;
        t.s2 = c.s2;
        t.s2_lds = c.s2_lds;
        float ms = 0.0f;
        e = run(t, &ms);
        if (e == hipSuccess && ms >= 0.0f && ms < best_t) {
            best_t = ms;
            best.s2 = c.s2;
            best.s2_lds = c.s2_lds;
        }
    }
    if (in) (void)hipFreeAsync(in, stream);
    if (out) (void)hipFreeAsync(out, stream);
    if (ws) (void)hipFreeAsync(ws, stream);
    const hipError_t es = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return tx::status_of(e);
    if (best_t < 0.0f) return TX_ENOTSUP;
    {
        std::lock_guard<std::mutex> lock(p->mu);
        p->tiles = best;
    }
    if (best_ms) *best_ms = best_t;
    return TX_OK;
}
