// Host side of a dedispersion plan: delay tables, sub-band partition, coarse
// groups and overlap (Sec. 2.3).  Pure host code; no device calls.
#include <algorithm>
#include <cmath>

#include "tx_internal.h"

#pragma clang fp contract(off)

namespace tx {

// D(DM, f) = floor(((k*DM) * (1/(f*f) - 1/(fref*fref))) / tsamp + 0.5), float64
// in exactly this order (Sec. 2.3, Eq. 1; half-up rounding to samples).
static int64_t delay64(double dm, double f, double fref, double tsamp) {
    volatile double inv_f2 = 1.0 / (f * f);
    volatile double inv_fref2 = 1.0 / (fref * fref);
    volatile double tau = (kDispersion * dm) * (inv_f2 - inv_fref2);
    volatile double x = tau / tsamp + 0.5;
    double fl = std::floor(x);
    if (!(fl < 9.0e18)) return INT64_MAX;
    return static_cast<int64_t>(fl);
}

int32_t delay_samples(double dm, double f, double fref, double tsamp) {
    return static_cast<int32_t>(delay64(dm, f, fref, tsamp));
}

// Coarse group size (see tx.h): g = 1 + floor((a_full / a_max) / 2), capped.
static int32_t group_rule(const std::vector<double>& f, int32_t nsub, int32_t ndm) {
    const int32_t nchan = static_cast<int32_t>(f.size());
    const int32_t m = nchan / nsub;
    double fref = *std::max_element(f.begin(), f.end());
    double fmin = *std::min_element(f.begin(), f.end());
    double a_full = 1.0 / (fmin * fmin) - 1.0 / (fref * fref);
    double a_max = 0.0;
    for (int32_t s = 0; s < nsub; ++s) {
        double hi = f[s * m], lo = f[s * m];
        for (int32_t c = s * m; c < (s + 1) * m; ++c) {
            hi = std::max(hi, f[c]);
            lo = std::min(lo, f[c]);
        }
        double a_s = 1.0 / (lo * lo) - 1.0 / (hi * hi);
        a_max = std::max(a_max, a_s);
    }
    if (m == 1 || !(a_max > 0.0)) return ndm;
    double ratio = a_full / a_max;
    double g = 1.0 + std::floor(ratio / 2.0);
    if (!(g < static_cast<double>(ndm))) return ndm;
    return std::max<int32_t>(1, static_cast<int32_t>(g));
}

// Automatic sub-band count: the divisor of nchan with at most 256 channels per
// sub-band that minimises the modelled time per output sample,
// N_c * N_f + kStage2AddCost * N_DM * nsub.  A second-stage addition costs
// about 2.5 first-stage ones on MI355X: the first stage sums 35 T byte-adds/s
// and the second 16 T adds/s on the paper-scale block, and the uneven
// 64-beam batch runs fastest at about the sub-band counts this weight picks.
constexpr double kStage2AddCost = 2.5;

static int32_t choose_nsub(const std::vector<double>& f, int32_t ndm) {
    const int32_t nchan = static_cast<int32_t>(f.size());
    int32_t best = -1;
    double best_cost = 0.0;
    for (int32_t ns = 1; ns <= nchan; ++ns) {
        if (nchan % ns != 0 || nchan / ns > kMaxChansPerSub) continue;
        int32_t g = group_rule(f, ns, ndm);
        int32_t ngroups = (ndm + g - 1) / g;
        double cost = static_cast<double>(ngroups) * nchan + kStage2AddCost * static_cast<double>(ndm) * ns;
        if (best < 0 || cost < best_cost) {
            best = ns;
            best_cost = cost;
        }
    }
    return best;
}

tx_status build_plan_host(const double* freqs, int32_t nchan, double tsamp, const double* dms,
                          int32_t ndm, int32_t nsub, int32_t dms_per_group, tx_plan_s* p) {
    if (!freqs || !dms || nchan < 1 || ndm < 1 || nsub < 0 || dms_per_group < 0) return TX_EINVAL;
    if (!(std::isfinite(tsamp) && tsamp > 0.0)) return TX_EINVAL;
    for (int32_t c = 0; c < nchan; ++c)
        if (!(std::isfinite(freqs[c]) && freqs[c] > 0.0)) return TX_EINVAL;
    for (int32_t i = 0; i < ndm; ++i) {
        if (!(std::isfinite(dms[i]) && dms[i] >= 0.0)) return TX_EINVAL;
        if (i > 0 && dms[i] < dms[i - 1]) return TX_EINVAL;
    }
    p->freqs.assign(freqs, freqs + nchan);
    p->dms.assign(dms, dms + ndm);
    if (nsub == 0) nsub = choose_nsub(p->freqs, ndm);
    if (nsub < 1 || nchan % nsub != 0 || nchan / nsub > kMaxChansPerSub) return TX_EINVAL;

    p->nchan = nchan;
    p->ndm = ndm;
    p->nsub = nsub;
    p->m = nchan / nsub;
    p->tsamp = tsamp;
    p->fref = *std::max_element(p->freqs.begin(), p->freqs.end());
    int32_t g = dms_per_group > 0 ? std::min(dms_per_group, ndm) : group_rule(p->freqs, nsub, ndm);
    p->g = g;
    p->ngroups = (ndm + g - 1) / g;
    const int32_t m = p->m, G = p->ngroups;

    std::vector<double> fsub(nsub);
    for (int32_t s = 0; s < nsub; ++s) {
        double hi = p->freqs[s * m];
        for (int32_t c = s * m; c < (s + 1) * m; ++c) hi = std::max(hi, p->freqs[c]);
        fsub[s] = hi;
    }
    // Every delay must fit the 32-bit tables (and stay far from overflow in
    // index arithmetic): the largest is D(max DM, lowest frequency).
    double fmin = *std::min_element(p->freqs.begin(), p->freqs.end());
    int64_t reach = delay64(p->dms[ndm - 1], fmin, p->fref, tsamp);
    if (reach >= kMaxDelay) return TX_EOVERFLOW;
    p->brute_reach = reach;

    p->coarse_chan.assign(static_cast<size_t>(G) * nchan, 0);
    p->coarse_sub.assign(static_cast<size_t>(G) * nsub, 0);
    p->fine_sub.assign(static_cast<size_t>(ndm) * nsub, 0);
    p->extent.assign(static_cast<size_t>(G) * nsub, 0);
    p->rel.assign(static_cast<size_t>(ndm) * nsub, 0);
    for (int32_t j = 0; j < G; ++j) {
        double c = p->dms[static_cast<size_t>(j) * g];
        for (int32_t ch = 0; ch < nchan; ++ch)
            p->coarse_chan[static_cast<size_t>(j) * nchan + ch] = delay_samples(c, p->freqs[ch], p->fref, tsamp);
        for (int32_t s = 0; s < nsub; ++s)
            p->coarse_sub[static_cast<size_t>(j) * nsub + s] = delay_samples(c, fsub[s], p->fref, tsamp);
    }
    int64_t max_off = 0, max_ext = 0;
    for (int32_t i = 0; i < ndm; ++i) {
        int32_t j = i / g;
        for (int32_t s = 0; s < nsub; ++s) {
            int32_t fs = delay_samples(p->dms[i], fsub[s], p->fref, tsamp);
            int32_t r = fs - p->coarse_sub[static_cast<size_t>(j) * nsub + s];
            p->fine_sub[static_cast<size_t>(i) * nsub + s] = fs;
            p->rel[static_cast<size_t>(i) * nsub + s] = r;
            int32_t& e = p->extent[static_cast<size_t>(j) * nsub + s];
            e = std::max(e, r);
            max_ext = std::max<int64_t>(max_ext, r);
        }
    }
    for (int32_t i = 0; i < ndm; ++i) {
        int32_t j = i / g;
        for (int32_t ch = 0; ch < nchan; ++ch) {
            int32_t s = ch / m;
            int64_t off = static_cast<int64_t>(p->coarse_chan[static_cast<size_t>(j) * nchan + ch]) +
                          p->rel[static_cast<size_t>(i) * nsub + s];
            max_off = std::max(max_off, off);
        }
    }
    p->max_extent = max_ext;
    p->overlap = std::max(max_off, reach);

    // Transposed tables for the kernels: a wave reads the delays of its
    // consecutive trials for one channel (or sub-band) from one row.  The
    // trial axis is padded with copies of the last trial.
    p->gpad = G + kTablePad;
    p->dT.assign(static_cast<size_t>(nchan) * p->gpad, 0);
    for (int32_t ch = 0; ch < nchan; ++ch)
        for (int32_t j = 0; j < p->gpad; ++j)
            p->dT[static_cast<size_t>(ch) * p->gpad + j] =
                p->coarse_chan[static_cast<size_t>(std::min(j, G - 1)) * nchan + ch];
    p->dpad = ndm + kTablePad;
    p->rT.assign(static_cast<size_t>(nsub) * p->dpad, 0);
    for (int32_t s = 0; s < nsub; ++s)
        for (int32_t i = 0; i < p->dpad; ++i)
            p->rT[static_cast<size_t>(s) * p->dpad + i] = p->rel[static_cast<size_t>(std::min(i, ndm - 1)) * nsub + s];
    return TX_OK;
}

int32_t plan_spread1(const tx_plan_s* p, int J) {
    std::lock_guard<std::mutex> lock(p->mu);
    for (auto& e : p->spread1_cache)
        if (e.first == J) return e.second;
    int32_t sp = 0;
    for (int32_t j0 = 0; j0 < p->ngroups; j0 += J) {
        const int32_t jl = std::min(j0 + J, p->ngroups) - 1;
        for (int32_t ch = 0; ch < p->nchan; ++ch)
            sp = std::max(sp, p->coarse_chan[static_cast<size_t>(jl) * p->nchan + ch] -
                                  p->coarse_chan[static_cast<size_t>(j0) * p->nchan + ch]);
    }
    p->spread1_cache.emplace_back(J, sp);
    return sp;
}

int32_t plan_spread2(const tx_plan_s* p, int iw) {
    std::lock_guard<std::mutex> lock(p->mu);
    for (auto& e : p->spread2_cache)
        if (e.first == iw) return e.second;
    int32_t sp = 0;
    for (int32_t j = 0; j < p->ngroups; ++j) {
        const int32_t iend = std::min((j + 1) * p->g, p->ndm);
        for (int32_t i0 = j * p->g; i0 < iend; i0 += iw) {
            const int32_t il = std::min(i0 + iw, iend) - 1;
            for (int32_t s = 0; s < p->nsub; ++s)
                sp = std::max(sp, p->rel[static_cast<size_t>(il) * p->nsub + s] -
                                      p->rel[static_cast<size_t>(i0) * p->nsub + s]);
        }
    }
    p->spread2_cache.emplace_back(iw, sp);
    return sp;
}

}  // namespace tx
