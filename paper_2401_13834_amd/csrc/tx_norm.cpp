// The C ABI of the normalised (floating-point) variant: per-channel weights
// from exact power sums (host), dedispersion of the normalised block, and the
// matched filter of float DM x time arrays (Sec. 2.1, 2.3, 2.4).
#include <cmath>
#include <cstring>

#include "tx_internal.h"

#pragma clang fp contract(off)

namespace {

tx_status check_plan(const tx_plan_s* p) {
    if (!p) return TX_EINVAL;
    if (!p->on_device) return TX_ESTATE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TX_EDEVICE;
    return dev == p->device ? TX_OK : TX_ESTATE;
}

// Widths of a float boxcar (validated as the integer path's).
tx_status fill_widths(const int32_t* widths, int32_t nw, int64_t nt, tx::BoxcarNormArgs* a) {
    tx::BoxcarArgs b{};
    const tx_status st = tx::boxcar_widths(widths, nw, nt, &b);
    if (st != TX_OK) return st;
    a->ne = b.ne;
    a->wmax = b.wmax;
    a->w_first = b.w_first;
    for (int k = 0; k < TX_MAX_WIDTHS; ++k) {
        a->widths[k] = b.widths[k];
        a->rsw[k] = b.rsw[k];
    }
    return TX_OK;
}

tx_status boxcar_norm(const float* d_dmt, int32_t ndm, int64_t nt, int64_t pitch, const int32_t* widths, int32_t nw,
                      double gamma, bool cands, tx_cand* d_out, int64_t cap, int64_t* d_count, double* d_snr,
                      int32_t* d_width, int64_t* d_time, hipStream_t stream, bool fixed = false, double mean = 0.0,
                      double sigma = 1.0) {
    if (ndm < 0 || nt < 1 || nt > TX_MAX_NT_BOXCAR || pitch < nt || (ndm > 0 && !d_dmt)) return TX_EINVAL;
    tx::BoxcarNormArgs a{};
    tx_status st = fill_widths(widths, nw, nt, &a);
    if (st != TX_OK) return st;
    const bool peaks = d_snr || d_width || d_time;
    if (peaks && !(d_snr && d_width && d_time)) return TX_EINVAL;
    if (cands && (!std::isfinite(gamma) || cap < 0 || !d_count || (cap > 0 && !d_out))) return TX_EINVAL;
    if (!cands && !peaks) return TX_EINVAL;
    a.y = d_dmt;
    a.pitch = pitch;
    a.ndm = ndm;
    a.nt = static_cast<int32_t>(nt);
    a.gamma = gamma;
    a.want_peaks = peaks ? 1 : 0;
    a.want_cands = cands ? 1 : 0;
    a.snr = d_snr;
    a.width = d_width;
    a.time = d_time;
    a.cands = d_out;
    a.cap = cap;
    a.count = reinterpret_cast<unsigned long long*>(d_count);
    a.fixed = fixed ? 1 : 0;
    a.fixed_mean = mean;
    a.fixed_sigma = sigma;
    return tx::status_of(tx::launch_boxcar_norm(a, stream));
}

}  // namespace

extern "C" {

tx_status tx_norm_weights(const uint64_t* sums, int32_t nchan, int64_t nt, int32_t weighting, float* scale,
                          float* offset) {
    if (!sums || !scale || !offset || nchan < 1 || nt < 1 || nt > (int64_t(1) << 32) ||
        (weighting != TX_WEIGHT_UNIT && weighting != TX_WEIGHT_INVERSE_VAR))
        return TX_EINVAL;
    for (int32_t c = 0; c < nchan; ++c) {
        const uint64_t s1 = sums[4 * static_cast<size_t>(c)], s2 = sums[4 * static_cast<size_t>(c) + 1];
        const unsigned __int128 n = static_cast<unsigned __int128>(nt);
        const unsigned __int128 a = n * s2, b = static_cast<unsigned __int128>(s1) * s1;
        if (b > a) return TX_EINVAL;                       // not the sums of one channel's samples
        const double mean = static_cast<double>(s1) / static_cast<double>(nt);
        const double var = static_cast<double>(a - b) / static_cast<double>(n * n);
        if (!(var > 0.0)) {
            scale[c] = 0.0f;
            offset[c] = 0.0f;
            continue;
        }
        const double w = weighting == TX_WEIGHT_UNIT ? 1.0 / std::sqrt(var) : 1.0 / var;
        scale[c] = static_cast<float>(w);
        offset[c] = static_cast<float>(w * mean);
    }
    return TX_OK;
}

tx_status tx_dedisperse_norm_ws_size(tx_plan_t p, int64_t nt, int64_t* bytes) {
    if (!p || !bytes || nt < 0) return TX_EINVAL;
    *bytes = nt == 0 ? 0 : tx::norm_geometry(p, nt).ws_bytes;
    return TX_OK;
}

tx_status tx_dedisperse_norm(tx_plan_t p, const uint8_t* d_in, int64_t in_pitch, int64_t nt, const float* d_scale,
                             const float* d_offset, float* d_out, int64_t out_pitch, hipStream_t stream) {
    tx_status st = check_plan(p);
    if (st != TX_OK) return st;
    if (nt < 0 || nt > (int64_t(1) << 30)) return TX_EINVAL;
    if (nt == 0) return TX_OK;
    if (!d_in || !d_out || !d_scale || !d_offset) return TX_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_in) & 15) || (in_pitch & 15) || in_pitch < nt + p->overlap) return TX_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_scale) & 3) || (reinterpret_cast<uintptr_t>(d_offset) & 3)) return TX_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_out) & 3) || out_pitch < nt) return TX_EINVAL;
    st = tx::retain_pool(p->device);
    if (st != TX_OK) return st;
    const tx::NormGeom g = tx::norm_geometry(p, nt);
    if (!g.ok) return TX_ENOTSUP;
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, static_cast<size_t>(g.ws_bytes), stream);
    if (e != hipSuccess) return tx::status_of(e);
    e = tx::launch_dedisperse_norm(p, g, d_in, in_pitch, nt, d_scale, d_offset, d_out, out_pitch,
                                   static_cast<float*>(ws), stream);
    const hipError_t f = hipFreeAsync(ws, stream);
    if (e != hipSuccess) return tx::status_of(e);
    return tx::status_of(f);
}

tx_status tx_boxcar_snr_f32(const float* d_dmt, int32_t ndm, int64_t nt, int64_t pitch, const int32_t* widths,
                            int32_t nw, double* d_snr, int32_t* d_width, int64_t* d_time, hipStream_t stream) {
    if (ndm > 0 && !(d_snr && d_width && d_time)) return TX_EINVAL;
    return boxcar_norm(d_dmt, ndm, nt, pitch, widths, nw, 0.0, false, nullptr, 0, nullptr, d_snr, d_width, d_time,
                       stream);
}

tx_status tx_boxcar_snr_fixed(const float* d_dmt, int32_t ndm, int64_t nt, int64_t pitch, const int32_t* widths,
                              int32_t nw, double mean, double sigma, double* d_snr, int32_t* d_width, int64_t* d_time,
                              hipStream_t stream) {
    if (ndm > 0 && !(d_snr && d_width && d_time)) return TX_EINVAL;
    if (!std::isfinite(mean) || !std::isfinite(sigma) || !(sigma > 0.0)) return TX_EINVAL;
    return boxcar_norm(d_dmt, ndm, nt, pitch, widths, nw, 0.0, false, nullptr, 0, nullptr, d_snr, d_width, d_time,
                       stream, true, mean, sigma);
}

tx_status tx_candidates_f32(const float* d_dmt, int32_t ndm, int64_t nt, int64_t pitch, const int32_t* widths,
                            int32_t nw, double gamma, tx_cand* d_out, int64_t cap, int64_t* d_count, double* d_snr,
                            int32_t* d_width, int64_t* d_time, hipStream_t stream) {
    return boxcar_norm(d_dmt, ndm, nt, pitch, widths, nw, gamma, true, d_out, cap, d_count, d_snr, d_width, d_time,
                       stream);
}

}  // extern "C"
