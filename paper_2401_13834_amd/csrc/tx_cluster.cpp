// Host side of the DM-time clustering (Sec. 2.5): the delay of every DM trial
// across the band (Eq. 1, in samples, unrounded) and, for a radius r, the
// range of DM trials whose delay lies within r of each trial.
#include <cmath>
#include <vector>

#include "tx_internal.h"

#pragma clang fp contract(off)

extern "C" {

tx_status tx_cluster(tx_plan_t p, const tx_cand* d_cands, int64_t n, double radius, int32_t min_pts,
                     tx_cand* d_sorted, int32_t* d_label, int64_t* d_rep, int64_t* d_nclusters, hipStream_t stream) {
    if (!p || n < 0 || n > INT32_MAX - 1 || !(radius > 0.0) || !(radius <= 1.0e6) || min_pts < 0 || !d_nclusters)
        return TX_EINVAL;
    if (n > 0 && (!d_cands || !d_sorted || !d_label || !d_rep)) return TX_EINVAL;
    if (!p->on_device) return TX_ESTATE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TX_EDEVICE;
    if (dev != p->device) return TX_ESTATE;
    tx_status st = tx::retain_pool(dev);
    if (st != TX_OK) return st;

    // x[d] = ((k DM_d) (1/f_lo^2 - 1/f_hi^2)) / tsamp, as the plan's delays
    // are formed but unrounded; DM trials are non-decreasing, so x is too.
    const int32_t ndm = p->ndm;
    double flo = p->freqs[0], fhi = p->freqs[0];
    for (double f : p->freqs) {
        flo = std::min(flo, f);
        fhi = std::max(fhi, f);
    }
    const double inv_lo = 1.0 / (flo * flo);
    const double inv_hi = 1.0 / (fhi * fhi);
    std::vector<double> x(ndm);
    for (int32_t d = 0; d < ndm; ++d) x[d] = ((tx::kDispersion * p->dms[d]) * (inv_lo - inv_hi)) / p->tsamp;
    // DM trials within r of each trial in delay: a contiguous range.
    std::vector<int32_t> lohi(2 * static_cast<size_t>(ndm));
    const double r2 = radius * radius;
    int32_t lo = 0, hi = 0;
    for (int32_t d = 0; d < ndm; ++d) {
        while ((x[d] - x[lo]) * (x[d] - x[lo]) > r2) ++lo;
        if (hi < d) hi = d;
        while (hi + 1 < ndm && (x[hi + 1] - x[d]) * (x[hi + 1] - x[d]) <= r2) ++hi;
        lohi[d] = lo;
        lohi[ndm + d] = hi;
    }
    void* buf = nullptr;
    const size_t xb = sizeof(double) * ndm, lb = sizeof(int32_t) * 2 * ndm;
    hipError_t e = hipMallocAsync(&buf, xb + lb, stream);
    if (e != hipSuccess) return tx::status_of(e);
    double* d_x = static_cast<double*>(buf);
    int32_t* d_lohi = reinterpret_cast<int32_t*>(static_cast<uint8_t*>(buf) + xb);
    e = hipMemcpyAsync(d_x, x.data(), xb, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_lohi, lohi.data(), lb, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = tx::launch_cluster(d_cands, n, ndm, d_x, d_lohi, d_lohi + ndm, radius, min_pts, d_sorted, d_label, d_rep,
                               d_nclusters, stream);
    // The host tables must outlive the copies.
    const hipError_t s = hipStreamSynchronize(stream);
    const hipError_t f = hipFreeAsync(buf, stream);
    if (e == hipSuccess) e = s;
    if (e == hipSuccess) e = f;
    return tx::status_of(e);
}

}  // extern "C"
