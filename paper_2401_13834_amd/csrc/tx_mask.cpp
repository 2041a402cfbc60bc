// Channel statistics and the narrow-band RFI mask (Sec. 2.2): the paper's
// skewness-kurtosis filter removes channels that are outliers in skewness and
// kurtosis across the band.  Host part: the decision from the exact power
// sums that tx_channel_power_sums computes on the device.
//
// Reading (the paper gives the rule's intent, not its constants): a
// channel's skewness g1 = m3 / m2^1.5 and kurtosis b2 = m4 / m2^2 (population
// central moments); over the channels with m2 > 0, a channel is an outlier in
// a statistic when |s - median| > threshold * 1.482602218505602 * MAD (median
// absolute deviation; with MAD = 0, any s != median); channels that are
// outliers in either statistic, or have m2 = 0, are masked.
#include <algorithm>
#include <cmath>
#include <vector>

#include "tx_internal.h"

#pragma clang fp contract(off)

namespace {

using i128 = __int128;

// Median of v (mean of the two middle values for an even count).
double median(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    const size_t n = v.size();
    return n % 2 ? v[n / 2] : (v[n / 2 - 1] + v[n / 2]) / 2.0;
}

// Outliers of s (indexed like `idx`) by the robust z rule.
void outliers(const std::vector<double>& s, double threshold, std::vector<bool>& out) {
    const double med = median(s);
    std::vector<double> dev(s.size());
    for (size_t i = 0; i < s.size(); ++i) dev[i] = std::fabs(s[i] - med);
    const double mad = median(dev);
    const double lim = threshold * (1.482602218505602 * mad);
    for (size_t i = 0; i < s.size(); ++i) out[i] = out[i] || (mad > 0.0 ? dev[i] > lim : dev[i] != 0.0);
}

}  // namespace

extern "C" {

tx_status tx_channel_power_sums(const uint8_t* d_in, int64_t in_pitch, int32_t nchan, int64_t nt, uint64_t* d_sums,
                                hipStream_t stream) {
    // sum x^4 < 2^64 for nt <= 2^32
    if (nchan < 1 || nt < 0 || nt > (int64_t(1) << 32) || !d_sums || (nt > 0 && (!d_in || in_pitch < nt)))
        return TX_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_in) & 15) || (in_pitch & 15) || (reinterpret_cast<uintptr_t>(d_sums) & 7))
        return TX_EINVAL;
    return tx::status_of(tx::launch_power_sums(d_in, in_pitch, nchan, nt, d_sums, stream));
}

tx_status tx_skf_mask(const uint64_t* sums, int32_t nchan, int64_t nt, double threshold, uint8_t* mask) {
    // n^3 sum x^4 and (sum x)^4 stay below 2^126 for nt <= 2^23
    if (!sums || !mask || nchan < 1 || nt < 1 || nt > (int64_t(1) << 23) || !(threshold > 0.0)) return TX_EINVAL;
    std::vector<int32_t> idx;
    std::vector<double> g1, b2;
    const i128 n = nt;
    for (int32_t c = 0; c < nchan; ++c) {
        const i128 s1 = sums[4 * c], s2 = sums[4 * c + 1], s3 = sums[4 * c + 2], s4 = sums[4 * c + 3];
        // n^2 m2, n^3 m3, n^4 m4 as exact integers
        const i128 M2 = n * s2 - s1 * s1;
        const i128 M3 = n * n * s3 - 3 * n * s1 * s2 + 2 * s1 * s1 * s1;
        const i128 M4 = n * n * n * s4 - 4 * n * n * s1 * s3 + 6 * n * s1 * s1 * s2 - 3 * s1 * s1 * s1 * s1;
        mask[c] = 0;
        if (M2 <= 0) continue;
        const double m2 = static_cast<double>(M2), m3 = static_cast<double>(M3), m4 = static_cast<double>(M4);
        idx.push_back(c);
        g1.push_back(m3 / (m2 * std::sqrt(m2)));
        b2.push_back(m4 / (m2 * m2));
    }
    if (idx.empty()) return TX_OK;
    std::vector<bool> bad(idx.size(), false);
    outliers(g1, threshold, bad);
    outliers(b2, threshold, bad);
    for (size_t i = 0; i < idx.size(); ++i) mask[idx[i]] = bad[i] ? 0 : 1;
    return TX_OK;
}

}  // extern "C"
