// The C ABI of libtx: argument checking, plan lifetime, scratch, launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "tx_internal.h"

using tx::kMaxChansPerSub;

namespace {

thread_local char t_last_error[256] = "";

tx_status from_hip(hipError_t e) { return tx::status_of(e); }

// Keep freed stream-ordered scratch in the device pool instead of handing it
// back to the driver at every synchronisation.
void release_device(tx_plan_s* p) {
    if (p->d_dT) (void)hipFree(p->d_dT);
    if (p->d_rT) (void)hipFree(p->d_rT);
    if (p->d_mask) (void)hipFree(p->d_mask);
    p->d_dT = nullptr;
    p->d_rT = nullptr;
    p->d_mask = nullptr;
    p->on_device = false;
}

tx_status upload(tx_plan_s* p) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TX_EDEVICE;
    const size_t n1 = p->dT.size() * sizeof(int32_t);
    const size_t n2 = p->rT.size() * sizeof(int32_t);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->d_dT), n1);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->d_rT), n2);
    if (e == hipSuccess) e = hipMemcpy(p->d_dT, p->dT.data(), n1, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_rT, p->rT.data(), n2, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release_device(p);
        return from_hip(e);
    }
    p->device = dev;
    p->on_device = true;
    return TX_OK;
}

tx::Tiles current_tiles(const tx_plan_s* p) { return tx::plan_tiles(p); }

tx_status check_device_plan(const tx_plan_s* p) {
    if (!p) return TX_EINVAL;
    if (!p->on_device) return TX_ESTATE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TX_EDEVICE;
    if (dev != p->device) return TX_ESTATE;
    return TX_OK;
}

tx_status check_dedisp_args(const tx_plan_s* p, const uint8_t* d_in, int64_t in_pitch, int64_t nt,
                            const int32_t* d_out, int64_t out_pitch) {
    if (nt < 0 || nt > (int64_t(1) << 30)) return TX_EINVAL;
    if (nt == 0) return TX_OK;
    if (!d_in || !d_out) return TX_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_in) & 15) || (in_pitch & 15)) return TX_EINVAL;
    if (in_pitch < nt + p->overlap) return TX_EINVAL;
    return tx::check_out_args(d_out, out_pitch, nt);
}

tx_status check_boxcar_args(const int32_t* d_dmt, int32_t ndm, int64_t nt, int64_t pitch, const int32_t* widths,
                            int32_t nw, tx::BoxcarArgs* a) {
    if (ndm < 0 || nt < 1 || nt > TX_MAX_NT_BOXCAR || pitch < nt) return TX_EINVAL;
    if (ndm > 0 && !d_dmt) return TX_EINVAL;
    const tx_status st = tx::boxcar_widths(widths, nw, nt, a);
    if (st != TX_OK) return st;
    a->y = d_dmt;
    a->pitch = pitch;
    a->ndm = ndm;
    a->nt = static_cast<int32_t>(nt);
    return TX_OK;
}

}  // namespace

void tx::note_error(hipError_t e) {
    std::snprintf(t_last_error, sizeof(t_last_error), "%s (%d)", hipGetErrorString(e), static_cast<int>(e));
}

void tx::note_message(const char* msg) { std::snprintf(t_last_error, sizeof(t_last_error), "%s", msg); }

tx_status tx::status_of(hipError_t e) {
    if (e == hipSuccess) return TX_OK;
    tx::note_error(e);
    if (e == hipErrorOutOfMemory) return TX_ENOMEM;
    return TX_EDEVICE;
}

tx::Tiles tx::plan_tiles(const tx_plan_s* p) {
    std::lock_guard<std::mutex> lock(p->mu);
    return p->tiles;
}

tx_status tx::retain_pool(int dev) {
    static std::mutex mu;
    static bool done[64] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (dev < 0 || dev >= 64) return TX_EDEVICE;
    if (done[dev]) return TX_OK;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) return TX_EDEVICE;
    uint64_t thr = UINT64_MAX;
    if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr) != hipSuccess) return TX_EDEVICE;
    done[dev] = true;
    return TX_OK;
}

tx_status tx::boxcar_widths(const int32_t* widths, int32_t nw, int64_t nt, tx::BoxcarArgs* a) {
    if (!widths || nw < 1 || nw > TX_MAX_WIDTHS) return TX_EINVAL;
    for (int32_t k = 0; k < nw; ++k) {
        if (widths[k] < 1 || widths[k] > TX_MAX_WIDTH) return TX_EINVAL;
        if (k > 0 && widths[k] <= widths[k - 1]) return TX_EINVAL;
    }
    int32_t copy[TX_MAX_WIDTHS];
    for (int32_t k = 0; k < nw; ++k) copy[k] = widths[k];
    tx::boxcar_fit(a, copy, nw, nt);
    return TX_OK;
}

void tx::boxcar_fit(tx::BoxcarArgs* a, const int32_t* widths, int32_t nw, int64_t nt) {
    int32_t ne = 0;
    while (ne < nw && widths[ne] <= nt) ++ne;
    const int32_t w_first = widths[0];
    int32_t src[TX_MAX_WIDTHS];
    for (int32_t k = 0; k < TX_MAX_WIDTHS; ++k) src[k] = ne > 0 ? widths[std::min(k, ne - 1)] : w_first;
    a->nw = nw;
    a->ne = ne;
    a->w_first = w_first;
    a->wmax = ne > 0 ? widths[ne - 1] : 0;
    for (int32_t k = 0; k < TX_MAX_WIDTHS; ++k) {
        a->widths[k] = src[k];
        a->rsw[k] = 1.0 / std::sqrt(static_cast<double>(src[k]));
    }
}

int tx::boxcar_nwt(int n) { return n <= 4 ? 4 : n <= 8 ? 8 : n <= 10 ? 10 : n <= 12 ? 12 : n <= 16 ? 16 : 32; }

tx_status tx::check_out_args(const int32_t* d_out, int64_t out_pitch, int64_t nt) {
    if (!d_out || (reinterpret_cast<uintptr_t>(d_out) & 7) || (out_pitch & 1) || out_pitch < nt) return TX_EINVAL;
    return TX_OK;
}

extern "C" {

const char* tx_last_error(void) { return t_last_error; }


const char* tx_status_str(tx_status s) {
    switch (s) {
        case TX_OK: return "TX_OK";
        case TX_EINVAL: return "TX_EINVAL";
        case TX_ENOMEM: return "TX_ENOMEM";
        case TX_EDEVICE: return "TX_EDEVICE";
        case TX_ESTATE: return "TX_ESTATE";
        case TX_EOVERFLOW: return "TX_EOVERFLOW";
        case TX_ENOTSUP: return "TX_ENOTSUP";
    }
    return "TX_UNKNOWN";
}

const char* tx_version(void) { return "libtx 0.1 gfx950"; }

tx_status tx_plan_ex(const double* freqs_mhz, int32_t nchan, double tsamp_s, const double* dms, int32_t ndm,
                     int32_t nsub, int32_t dms_per_group, uint32_t flags, tx_plan_t* out) {
    if (!out) return TX_EINVAL;
    *out = nullptr;
    if (flags & ~TX_PLAN_HOST_ONLY) return TX_EINVAL;
    tx_plan_s* p = new (std::nothrow) tx_plan_s();
    if (!p) return TX_ENOMEM;
    tx_status st;
    try {
        st = tx::build_plan_host(freqs_mhz, nchan, tsamp_s, dms, ndm, nsub, dms_per_group, p);
    } catch (const std::bad_alloc&) {
        st = TX_ENOMEM;
    }
    if (st == TX_OK && !(flags & TX_PLAN_HOST_ONLY)) st = upload(p);
    if (st != TX_OK) {
        delete p;
        return st;
    }
    *out = p;
    return TX_OK;
}

tx_status tx_plan(const double* freqs_mhz, int32_t nchan, double tsamp_s, const double* dms, int32_t ndm,
                  int32_t nsub, tx_plan_t* out) {
    return tx_plan_ex(freqs_mhz, nchan, tsamp_s, dms, ndm, nsub, 0, 0u, out);
}

tx_status tx_plan_query(tx_plan_t p, tx_plan_info* i) {
    if (!p || !i) return TX_EINVAL;
    i->nchan = p->nchan;
    i->ndm = p->ndm;
    i->nsub = p->nsub;
    i->chans_per_sub = p->m;
    i->g = p->g;
    i->ngroups = p->ngroups;
    i->overlap = p->overlap;
    i->max_extent = p->max_extent;
    i->brute_reach = p->brute_reach;
    i->fref_mhz = p->fref;
    i->tsamp_s = p->tsamp;
    i->on_device = p->on_device ? 1 : 0;
    i->device = p->on_device ? p->device : -1;
    return TX_OK;
}

tx_status tx_plan_offsets(tx_plan_t p, int32_t* host_off) {
    if (!p || !host_off) return TX_EINVAL;
    for (int32_t i = 0; i < p->ndm; ++i) {
        const int32_t j = i / p->g;
        for (int32_t ch = 0; ch < p->nchan; ++ch) {
            const int32_t s = ch / p->m;
            host_off[static_cast<size_t>(i) * p->nchan + ch] =
                p->coarse_chan[static_cast<size_t>(j) * p->nchan + ch] + p->rel[static_cast<size_t>(i) * p->nsub + s];
        }
    }
    return TX_OK;
}

tx_status tx_plan_tables(tx_plan_t p, int32_t* coarse_chan, int32_t* coarse_sub, int32_t* fine_sub,
                         int32_t* extent) {
    if (!p) return TX_EINVAL;
    if (coarse_chan) std::memcpy(coarse_chan, p->coarse_chan.data(), p->coarse_chan.size() * sizeof(int32_t));
    if (coarse_sub) std::memcpy(coarse_sub, p->coarse_sub.data(), p->coarse_sub.size() * sizeof(int32_t));
    if (fine_sub) std::memcpy(fine_sub, p->fine_sub.data(), p->fine_sub.size() * sizeof(int32_t));
    if (extent) std::memcpy(extent, p->extent.data(), p->extent.size() * sizeof(int32_t));
    return TX_OK;
}

tx_status tx_plan_delays(tx_plan_t p, double dm, int32_t* host_delay) {
    if (!p || !host_delay || !(std::isfinite(dm) && dm >= 0.0)) return TX_EINVAL;
    double fmin = *std::min_element(p->freqs.begin(), p->freqs.end());
    double reach = tx::kDispersion * dm * (1.0 / (fmin * fmin) - 1.0 / (p->fref * p->fref)) / p->tsamp;
    if (!(reach < static_cast<double>(tx::kMaxDelay))) return TX_EOVERFLOW;
    for (int32_t c = 0; c < p->nchan; ++c) host_delay[c] = tx::delay_samples(dm, p->freqs[c], p->fref, p->tsamp);
    return TX_OK;
}

tx_status tx_pool_trim(void) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TX_EDEVICE;
    hipMemPool_t pool;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipDeviceGetDefaultMemPool(&pool, dev);
    if (e == hipSuccess) e = hipMemPoolTrimTo(pool, 0);
    return from_hip(e);
}

tx_status tx_plan_destroy(tx_plan_t p) {
    if (!p) return TX_OK;
    release_device(p);
    delete p;
    return TX_OK;
}

tx_status tx_dedisperse_ws_size(tx_plan_t p, int64_t nt, int64_t* bytes) {
    if (!p || !bytes || nt < 0) return TX_EINVAL;
    if (nt == 0) {
        *bytes = 0;
        return TX_OK;
    }
    const tx::DedispGeom g = tx::dedisp_geometry(p, nt, current_tiles(p));
    if (!g.ok) return TX_ENOTSUP;                  // as tx_dedisperse would answer
    *bytes = g.ws_bytes;
    return TX_OK;
}

tx_status tx_dedisperse_ws(tx_plan_t p, const uint8_t* d_in, int64_t in_pitch, int64_t nt, int32_t* d_out,
                           int64_t out_pitch, void* d_ws, int64_t ws_bytes, hipStream_t stream) {
    tx_status st = check_device_plan(p);
    if (st != TX_OK) return st;
    st = check_dedisp_args(p, d_in, in_pitch, nt, d_out, out_pitch);
    if (st != TX_OK || nt == 0) return st;
    const tx::DedispGeom geo = tx::dedisp_geometry(p, nt, current_tiles(p));
    if (!geo.ok) return TX_ENOTSUP;
    if (!d_ws || ws_bytes < geo.ws_bytes || (reinterpret_cast<uintptr_t>(d_ws) & 255)) return TX_EINVAL;
    return from_hip(tx::launch_dedisperse(p, geo, d_in, in_pitch, nt, d_out, out_pitch,
                                          static_cast<uint16_t*>(d_ws), stream));
}

tx_status tx_dedisperse_noalloc(tx_plan_t p, const uint8_t* d_in, int64_t in_pitch, int64_t nt, int32_t* d_out,
                                int64_t out_pitch, hipStream_t stream) {
    tx_status st = check_device_plan(p);
    if (st != TX_OK) return st;
    st = check_dedisp_args(p, d_in, in_pitch, nt, d_out, out_pitch);
    if (st != TX_OK || nt == 0) return st;
    int64_t need = 0;
    const hipError_t e = tx::launch_dedisperse_noalloc(p, current_tiles(p), d_in, in_pitch, nt, d_out, out_pitch,
                                                       stream, p->device, &need);
    if (e == hipErrorInvalidValue && need != 0) {
        char msg[200];
        if (need > 0)
            std::snprintf(msg, sizeof(msg),
                          "tx_dedisperse_noalloc: one chunk of this plan's first-stage series needs %lld bytes, "
                          "more than the %lld-byte scratch", static_cast<long long>(need),
                          static_cast<long long>(TX_NOALLOC_SCRATCH_BYTES));
        else
            std::snprintf(msg, sizeof(msg), "tx_dedisperse_noalloc: no tile of this plan fits the device's LDS");
        tx::note_message(msg);
        return TX_ENOTSUP;
    }
    return from_hip(e);
}

tx_status tx_dedisperse(tx_plan_t p, const uint8_t* d_in, int64_t in_pitch, int64_t nt, int32_t* d_out,
                        int64_t out_pitch, hipStream_t stream) {
    tx_status st = check_device_plan(p);
    if (st != TX_OK) return st;
    st = check_dedisp_args(p, d_in, in_pitch, nt, d_out, out_pitch);
    if (st != TX_OK || nt == 0) return st;
    st = tx::retain_pool(p->device);
    if (st != TX_OK) return st;
    const tx::DedispGeom geo = tx::dedisp_geometry(p, nt, current_tiles(p));
    if (!geo.ok) return TX_ENOTSUP;
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, static_cast<size_t>(geo.ws_bytes), stream);
    if (e != hipSuccess) return from_hip(e);
    e = tx::launch_dedisperse(p, geo, d_in, in_pitch, nt, d_out, out_pitch, static_cast<uint16_t*>(ws), stream);
    hipError_t f = hipFreeAsync(ws, stream);
    if (e != hipSuccess) return from_hip(e);
    return from_hip(f);
}

tx_status tx_plan_set_mask(tx_plan_t p, const uint8_t* mask) {
    if (!p) return TX_EINVAL;
    tx_status st = check_device_plan(p);
    if (st != TX_OK) return st;
    // Work already queued may still read the old mask.
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return from_hip(e);
    bool keep_all = true;
    if (mask)
        for (int32_t c = 0; c < p->nchan; ++c) keep_all = keep_all && mask[c] != 0;
    if (keep_all) {
        if (p->d_mask) (void)hipFree(p->d_mask);
        p->d_mask = nullptr;
        p->mask.clear();
        return TX_OK;
    }
    if (!p->d_mask) {
        e = hipMalloc(reinterpret_cast<void**>(&p->d_mask), static_cast<size_t>(p->nchan));
        if (e != hipSuccess) {
            p->d_mask = nullptr;
            return from_hip(e);
        }
    }
    p->mask.assign(mask, mask + p->nchan);
    for (uint8_t& m : p->mask) m = m ? 1 : 0;
    e = hipMemcpy(p->d_mask, p->mask.data(), static_cast<size_t>(p->nchan), hipMemcpyHostToDevice);
    return from_hip(e);
}

tx_status tx_plan_get_mask(tx_plan_t p, uint8_t* mask) {
    if (!p || !mask) return TX_EINVAL;
    for (int32_t c = 0; c < p->nchan; ++c) mask[c] = p->mask.empty() ? 1 : p->mask[c];
    return TX_OK;
}

tx_status tx_transpose_tf(const uint8_t* d_tf, int64_t tf_pitch, int32_t nchan, int64_t nt, uint8_t* d_ft,
                          int64_t ft_pitch, hipStream_t stream) {
    if (nchan < 1 || nt < 0 || nt > (int64_t(1) << 40) || tf_pitch < nchan || ft_pitch < nt) return TX_EINVAL;
    if (nt == 0) return TX_OK;
    if (!d_tf || !d_ft || (reinterpret_cast<uintptr_t>(d_tf) & 15) || (reinterpret_cast<uintptr_t>(d_ft) & 15) ||
        (tf_pitch & 15) || (ft_pitch & 15))
        return TX_EINVAL;
    return from_hip(tx::launch_transpose_tf(d_tf, tf_pitch, nchan, nt, d_ft, ft_pitch, stream));
}

tx_status tx_tile_variants(int32_t stage, int32_t* count) {
    if (!count || (stage != 1 && stage != 2)) return TX_EINVAL;
    *count = stage == 1 ? tx::stage1_variant_count() : tx::stage2_variant_count();
    return TX_OK;
}

tx_status tx_tile_variant_info(int32_t stage, int32_t variant, int32_t* outputs_per_tile, int32_t* trials_per_wave) {
    if (!outputs_per_tile || !trials_per_wave) return TX_EINVAL;
    if (stage == 1 && variant >= 0 && variant < tx::stage1_variant_count()) {
        const tx::Stage1Variant v = tx::stage1_variant(variant);
        *outputs_per_tile = 256 * v.q;
        *trials_per_wave = v.jw;
        return TX_OK;
    }
    if (stage == 2 && variant >= 0 && variant < tx::stage2_variant_count()) {
        *outputs_per_tile = 512 * tx::stage2_variant(variant).q;
        *trials_per_wave = 0;
        return TX_OK;
    }
    return TX_EINVAL;
}

tx_status tx_plan_get_tiles(tx_plan_t p, tx_tiles* t) {
    if (!p || !t) return TX_EINVAL;
    const tx::Tiles c = current_tiles(p);
    t->stage1 = c.s1;
    t->stage1_lds = c.s1_lds;
    t->stage2 = c.s2;
    t->stage2_lds = c.s2_lds;
    return TX_OK;
}

tx_status tx_plan_resolved_tiles(tx_plan_t p, int64_t nt, tx_tiles* t) {
    if (!p || !t || nt < 0) return TX_EINVAL;
    const tx::Tiles c = tx::dedisp_geometry(p, nt, current_tiles(p)).tiles;
    t->stage1 = c.s1;
    t->stage1_lds = c.s1_lds;
    t->stage2 = c.s2;
    t->stage2_lds = c.s2_lds;
    return TX_OK;
}

tx_status tx_plan_set_tiles(tx_plan_t p, const tx_tiles* t) {
    if (!p || !t) return TX_EINVAL;
    if (t->stage1 < -1 || t->stage1 >= tx::stage1_variant_count()) return TX_EINVAL;
    if (t->stage2 < -1 || t->stage2 >= tx::stage2_variant_count()) return TX_EINVAL;
    if (t->stage1_lds < 0 || t->stage1_lds > tx::kMaxLds || t->stage2_lds < 0 || t->stage2_lds > tx::kMaxLds)
        return TX_EINVAL;
    std::lock_guard<std::mutex> lock(p->mu);
    p->tiles.s1 = t->stage1;
    p->tiles.s1_lds = t->stage1_lds;
    p->tiles.s2 = t->stage2;
    p->tiles.s2_lds = t->stage2_lds;
    return TX_OK;
}

tx_status tx_candidates(const int32_t* d_dmt, int32_t ndm, int64_t nt, int64_t pitch, const int32_t* widths,
                        int32_t nw, double gamma, tx_cand* d_out, int64_t cap, int64_t* d_count, double* d_snr,
                        int32_t* d_width, int64_t* d_time, hipStream_t stream) {
    tx::BoxcarArgs a{};
    tx_status st = check_boxcar_args(d_dmt, ndm, nt, pitch, widths, nw, &a);
    if (st != TX_OK) return st;
    if (!std::isfinite(gamma) || cap < 0 || !d_count || (cap > 0 && !d_out)) return TX_EINVAL;
    const bool peaks = d_snr || d_width || d_time;
    if (peaks && !(d_snr && d_width && d_time)) return TX_EINVAL;
    a.gamma = gamma;
    a.want_cands = 1;
    a.want_peaks = peaks ? 1 : 0;
    a.snr = d_snr;
    a.width = d_width;
    a.time = d_time;
    a.cands = d_out;
    a.cap = cap;
    a.count = reinterpret_cast<unsigned long long*>(d_count);
    return from_hip(tx::launch_boxcar(a, stream));
}

tx_status tx_boxcar_snr(const int32_t* d_dmt, int32_t ndm, int64_t nt, int64_t pitch, const int32_t* widths,
                        int32_t nw, double* d_snr, int32_t* d_width, int64_t* d_time, hipStream_t stream) {
    tx::BoxcarArgs a{};
    tx_status st = check_boxcar_args(d_dmt, ndm, nt, pitch, widths, nw, &a);
    if (st != TX_OK) return st;
    if (ndm > 0 && !(d_snr && d_width && d_time)) return TX_EINVAL;
    a.gamma = 0.0;
    a.want_cands = 0;
    a.want_peaks = 1;
    a.snr = d_snr;
    a.width = d_width;
    a.time = d_time;
    return from_hip(tx::launch_boxcar(a, stream));
}

}  // extern "C"
