// Dedispersion plans in DM ranges (Sec. 2.3): because intra-channel smearing
// exceeds the native sampling time at high DM, each DM range dedisperses the
// block downsampled in time by its own factor, with its own plan at the
// coarser sampling time, all in one call.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "tx_internal.h"

struct tx_ranges_s {
    std::vector<tx_plan_s*> plans;     // borrowed
    std::vector<int32_t> factors;
    int device = -1;
    int32_t nchan = 0;
};

namespace {

bool power_of_two_upto64(int32_t k) { return k >= 1 && k <= 64 && (k & (k - 1)) == 0; }

// Input samples one block of nt full-rate samples needs (nt a multiple of
// every factor), or -1.
int64_t input_len(const tx_ranges_s* r, int64_t nt) {
    int64_t need = 0;
    for (size_t i = 0; i < r->plans.size(); ++i) {
        const int64_t k = r->factors[i];
        if (nt % k) return -1;
        need = std::max(need, k * (nt / k + r->plans[i]->overlap));
    }
    return need;
}

}  // namespace

extern "C" {

tx_status tx_ranges_create(const tx_plan_t* plans, const int32_t* factors, int32_t n, tx_ranges_t* out) {
    if (!plans || !factors || !out || n < 1 || n > 64) return TX_EINVAL;
    *out = nullptr;
    const tx_plan_s* p0 = plans[0];
    if (!p0 || !power_of_two_upto64(factors[0])) return TX_EINVAL;
    const double base = p0->tsamp / factors[0];
    for (int32_t i = 0; i < n; ++i) {
        const tx_plan_s* p = plans[i];
        if (!p || !power_of_two_upto64(factors[i])) return TX_EINVAL;
        if (!p->on_device || p->device != p0->device) return TX_ESTATE;
        // Same channels; sampling time = base * factor.
        if (p->freqs != p0->freqs) return TX_EINVAL;
        if (std::fabs(p->tsamp - base * factors[i]) > 1e-9 * p->tsamp) return TX_EINVAL;
    }
    tx_ranges_s* r = new (std::nothrow) tx_ranges_s();
    if (!r) return TX_ENOMEM;
    r->plans.assign(plans, plans + n);
    r->factors.assign(factors, factors + n);
    r->device = p0->device;
    r->nchan = p0->nchan;
    *out = r;
    return TX_OK;
}

tx_status tx_ranges_input_len(tx_ranges_t r, int64_t nt, int64_t* need) {
    if (!r || !need || nt < 0) return TX_EINVAL;
    const int64_t v = input_len(r, nt);
    if (v < 0) return TX_EINVAL;
    *need = v;
    return TX_OK;
}

tx_status tx_ranges_dedisperse(tx_ranges_t r, const uint8_t* d_in, int64_t in_pitch, int64_t nt,
                               int32_t* const* d_outs, const int64_t* out_pitches, hipStream_t stream) {
    if (!r || !d_in || !d_outs || !out_pitches || nt < 0) return TX_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TX_EDEVICE;
    if (dev != r->device) return TX_ESTATE;
    const int64_t need = input_len(r, nt);
    if (need < 0 || in_pitch < need) return TX_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_in) & 15) || (in_pitch & 15)) return TX_EINVAL;
    const size_t n = r->plans.size();
    for (size_t i = 0; i < n; ++i) {
        const tx_status st = tx::check_out_args(d_outs[i], out_pitches[i], nt / r->factors[i]);
        if (st != TX_OK) return st;
    }
    if (nt == 0) return TX_OK;
    tx_status st = tx::retain_pool(dev);
    if (st != TX_OK) return st;

    // One downsampled copy per distinct factor > 1, long enough for every
    // range that uses it.
    std::vector<int32_t> ks;
    for (int32_t k : r->factors)
        if (k > 1 && std::find(ks.begin(), ks.end(), k) == ks.end()) ks.push_back(k);
    std::vector<void*> bufs(ks.size(), nullptr);
    std::vector<int64_t> pitches(ks.size(), 0);
    hipError_t e = hipSuccess;
    for (size_t b = 0; b < ks.size() && e == hipSuccess; ++b) {
        int64_t len = 0;
        for (size_t i = 0; i < n; ++i)
            if (r->factors[i] == ks[b]) len = std::max(len, nt / ks[b] + r->plans[i]->overlap);
        pitches[b] = (len + 255) / 256 * 256;
        e = hipMallocAsync(&bufs[b], static_cast<size_t>(pitches[b]) * r->nchan, stream);
        if (e == hipSuccess)
            e = tx::launch_downsample(d_in, in_pitch, r->nchan, len, ks[b], static_cast<uint8_t*>(bufs[b]),
                                      pitches[b], stream);
    }
    // Each range: its own plan on its (downsampled) copy.
    for (size_t i = 0; i < n && e == hipSuccess; ++i) {
        const tx_plan_s* p = r->plans[i];
        const int32_t k = r->factors[i];
        const int64_t nt_r = nt / k;
        if (nt_r == 0) continue;
        const uint8_t* in = d_in;
        int64_t pitch = in_pitch;
        if (k > 1) {
            const size_t b = static_cast<size_t>(std::find(ks.begin(), ks.end(), k) - ks.begin());
            in = static_cast<const uint8_t*>(bufs[b]);
            pitch = pitches[b];
        }
        const tx::DedispGeom geo = tx::dedisp_geometry(p, nt_r, tx::plan_tiles(p));
        if (!geo.ok) {
            st = TX_ENOTSUP;
            break;
        }
        void* ws = nullptr;
        e = hipMallocAsync(&ws, static_cast<size_t>(geo.ws_bytes), stream);
        if (e != hipSuccess) break;
        e = tx::launch_dedisperse(p, geo, in, pitch, nt_r, d_outs[i], out_pitches[i], static_cast<uint16_t*>(ws),
                                  stream);
        const hipError_t f = hipFreeAsync(ws, stream);
        if (e == hipSuccess) e = f;
    }
    for (void* b : bufs)
        if (b) (void)hipFreeAsync(b, stream);
    if (st != TX_OK) return st;
    return tx::status_of(e);
}

tx_status tx_downsample(const uint8_t* d_in, int64_t in_pitch, int32_t nchan, int64_t nt_out, int32_t k,
                        uint8_t* d_out, int64_t out_pitch, hipStream_t stream) {
    if (nchan < 1 || nt_out < 0 || !power_of_two_upto64(k) || nt_out > (int64_t(1) << 36)) return TX_EINVAL;
    if (nt_out == 0) return TX_OK;
    if (!d_in || !d_out || in_pitch < k * nt_out || out_pitch < nt_out) return TX_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_in) & 15) || (reinterpret_cast<uintptr_t>(d_out) & 15) || (in_pitch & 15) ||
        (out_pitch & 15))
        return TX_EINVAL;
    return tx::status_of(tx::launch_downsample(d_in, in_pitch, nchan, nt_out, k, d_out, out_pitch, stream));
}

tx_status tx_ranges_destroy(tx_ranges_t r) {
    delete r;
    return TX_OK;
}

}  // extern "C"
