/*
 * C oracle for sub-band dedispersion and the boxcar matched filter.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests (against the NumPy oracle and
 * brute force) and by the CPU-baseline leg of the benchmark.  Nothing in the
 * product path links or loads it, and it shares no code with the HIP path.
 *
 * A second, independent restatement of the same definitions as the NumPy
 * oracle, in the paper's order, with OpenMP over independent outputs:
 *   - integer delays D(DM, f) = floor(((k DM) (1/f^2 - 1/fref^2)) / tsamp + 0.5)
 *     (Sec. 2.3, Eq. 1; float64 in this order, no contraction), fref = the
 *     highest channel;
 *   - brute force Y[i][t] = sum_ch x[ch][t + D(dm_i, f_ch)];
 *   - sub-band method (Sec. 2.3): equal contiguous sub-bands, each referenced
 *     to its highest channel; groups of g consecutive fine trials whose coarse
 *     DM is the first trial; g = 1 + floor((a_full / a_max) / 2) unless given;
 *     stage 1  B[j][s][u] = sum_{ch in s} x[ch][u + D(c_j, f_ch)]
 *     stage 2  Y[i][t] = sum_s B[j][s][t + D(dm_i, f_s) - D(c_j, f_s)];
 *   - per-row statistics: c = floor(sum/T), Q = sum (y - c)^2, r = sum - T c,
 *     var = Q/T - (r/T)^2, inv_d = 1 / (sqrt(var) T) (Sec. 2.4);
 *   - boxcar S/N of the window [t, t + w): ((T S - w sum) inv_d) (1/sqrt(w))
 *     (Sec. 2.4, Eq. 5 with the block mean removed), peak per row (earliest
 *     start of the largest sum per width, largest S/N across widths, ties to
 *     the smaller width) and the thresholded DM-time points (Sec. 2.5).
 * Integer sums are exact (int64).  Built with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

static const double K_DM = 4.148808e3;

static int64_t delay(double dm, double f, double fref, double tsamp) {
    const double inv_f2 = 1.0 / (f * f);
    const double inv_fref2 = 1.0 / (fref * fref);
    const double tau = (K_DM * dm) * (inv_f2 - inv_fref2);
    return (int64_t)floor(tau / tsamp + 0.5);
}

static double max_of(const double* v, int n) {
    double m = v[0];
    for (int k = 1; k < n; ++k)
        if (v[k] > m) m = v[k];
    return m;
}

static double min_of(const double* v, int n) {
    double m = v[0];
    for (int k = 1; k < n; ++k)
        if (v[k] < m) m = v[k];
    return m;
}

int txo_group_rule(const double* freqs, int nchan, int nsub, int ndm) {
    const int m = nchan / nsub;
    const double fref = max_of(freqs, nchan), fmin = min_of(freqs, nchan);
    const double a_full = 1.0 / (fmin * fmin) - 1.0 / (fref * fref);
    double a_max = 0.0;
    for (int s = 0; s < nsub; ++s) {
        const double hi = max_of(freqs + s * m, m), lo = min_of(freqs + s * m, m);
        const double a_s = 1.0 / (lo * lo) - 1.0 / (hi * hi);
        if (a_s > a_max) a_max = a_s;
    }
    if (m == 1 || !(a_max > 0.0)) return ndm;
    int g = 1 + (int)floor((a_full / a_max) / 2.0);
    if (g < 1) g = 1;
    if (g > ndm) g = ndm;
    return g;
}

/* Tables of the sub-band plan.  d_cc [ngroups][nchan] = D(c_j, f_ch),
 * d_cs [ngroups][nsub] = D(c_j, f_s), d_fs [ndm][nsub] = D(dm_i, f_s);
 * *overlap = max(max_{i,ch} off(i, ch), D(dm_max, f_min)). */
int txo_plan_tables(const double* freqs, int nchan, double tsamp, const double* dms, int ndm, int nsub, int g,
                    int64_t* d_cc, int64_t* d_cs, int64_t* d_fs, int64_t* overlap) {
    if (nchan < 1 || ndm < 1 || nsub < 1 || nchan % nsub != 0 || g < 1) return -1;
    const int m = nchan / nsub;
    const int ngroups = (ndm + g - 1) / g;
    const double fref = max_of(freqs, nchan);
    double* fsub = malloc(sizeof(double) * nsub);
    if (!fsub) return -2;
    for (int s = 0; s < nsub; ++s) fsub[s] = max_of(freqs + s * m, m);
    for (int j = 0; j < ngroups; ++j) {
        const double c = dms[j * g];
        for (int ch = 0; ch < nchan; ++ch) d_cc[(int64_t)j * nchan + ch] = delay(c, freqs[ch], fref, tsamp);
        for (int s = 0; s < nsub; ++s) d_cs[(int64_t)j * nsub + s] = delay(c, fsub[s], fref, tsamp);
    }
    for (int i = 0; i < ndm; ++i)
        for (int s = 0; s < nsub; ++s) d_fs[(int64_t)i * nsub + s] = delay(dms[i], fsub[s], fref, tsamp);
    int64_t o = delay(dms[ndm - 1], min_of(freqs, nchan), fref, tsamp);
    for (int i = 0; i < ndm; ++i) {
        const int j = i / g;
        for (int ch = 0; ch < nchan; ++ch) {
            const int s = ch / m;
            const int64_t off = d_cc[(int64_t)j * nchan + ch] + d_fs[(int64_t)i * nsub + s] - d_cs[(int64_t)j * nsub + s];
            if (off > o) o = off;
        }
    }
    *overlap = o;
    free(fsub);
    return 0;
}

/* Brute force: x is nchan rows of >= nt + D(dm_max, f_min) samples. */
int txo_dedisperse_brute(const double* freqs, int nchan, double tsamp, const double* dms, int ndm, const uint8_t* x,
                         int64_t x_pitch, int64_t nt, int32_t* y, int64_t y_pitch, int nthreads) {
    const double fref = max_of(freqs, nchan);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int i = 0; i < ndm; ++i) {
        int32_t* out = y + (int64_t)i * y_pitch;
        for (int64_t t = 0; t < nt; ++t) out[t] = 0;
        for (int ch = 0; ch < nchan; ++ch) {
            const uint8_t* row = x + (int64_t)ch * x_pitch + delay(dms[i], freqs[ch], fref, tsamp);
            for (int64_t t = 0; t < nt; ++t) out[t] += row[t];
        }
    }
    return 0;
}

/* Two stages (g = 0: the rule). */
int txo_dedisperse_subband(const double* freqs, int nchan, double tsamp, const double* dms, int ndm, int nsub, int g,
                           const uint8_t* x, int64_t x_pitch, int64_t nt, int32_t* y, int64_t y_pitch, int nthreads) {
    if (nchan < 1 || nsub < 1 || nchan % nsub != 0) return -1;
    if (g <= 0) g = txo_group_rule(freqs, nchan, nsub, ndm);
    const int m = nchan / nsub;
    const int ngroups = (ndm + g - 1) / g;
    int64_t* d_cc = malloc(sizeof(int64_t) * (size_t)ngroups * nchan);
    int64_t* d_cs = malloc(sizeof(int64_t) * (size_t)ngroups * nsub);
    int64_t* d_fs = malloc(sizeof(int64_t) * (size_t)ndm * nsub);
    int64_t* ext = malloc(sizeof(int64_t) * (size_t)ngroups * nsub);
    int64_t* boff = malloc(sizeof(int64_t) * ((size_t)ngroups * nsub + 1));
    if (!d_cc || !d_cs || !d_fs || !ext || !boff) return -2;
    int64_t overlap = 0;
    int rc = txo_plan_tables(freqs, nchan, tsamp, dms, ndm, nsub, g, d_cc, d_cs, d_fs, &overlap);
    if (rc) return rc;
    /* extent of each first-stage series: max over the group's trials of
     * D(dm_i, f_s) - D(c_j, f_s) */
    boff[0] = 0;
    for (int j = 0; j < ngroups; ++j)
        for (int s = 0; s < nsub; ++s) {
            int64_t e = 0;
            for (int i = j * g; i < ndm && i < (j + 1) * g; ++i) {
                const int64_t d = d_fs[(int64_t)i * nsub + s] - d_cs[(int64_t)j * nsub + s];
                if (d > e) e = d;
            }
            ext[(int64_t)j * nsub + s] = e;
            boff[(int64_t)j * nsub + s + 1] = boff[(int64_t)j * nsub + s] + nt + e;
        }
    int32_t* B = malloc(sizeof(int32_t) * (size_t)boff[(int64_t)ngroups * nsub]);
    if (!B) return -2;
    /* stage 1: every sub-band at every coarse DM */
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t js = 0; js < (int64_t)ngroups * nsub; ++js) {
        const int j = (int)(js / nsub), s = (int)(js % nsub);
        int32_t* b = B + boff[js];
        const int64_t n = nt + ext[js];
        for (int64_t u = 0; u < n; ++u) b[u] = 0;
        for (int ch = s * m; ch < (s + 1) * m; ++ch) {
            const uint8_t* row = x + (int64_t)ch * x_pitch + d_cc[(int64_t)j * nchan + ch];
            for (int64_t u = 0; u < n; ++u) b[u] += row[u];
        }
    }
    /* stage 2: every fine trial from its group's sub-band series */
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int i = 0; i < ndm; ++i) {
        const int j = i / g;
        int32_t* out = y + (int64_t)i * y_pitch;
        for (int64_t t = 0; t < nt; ++t) out[t] = 0;
        for (int s = 0; s < nsub; ++s) {
            const int64_t e = d_fs[(int64_t)i * nsub + s] - d_cs[(int64_t)j * nsub + s];
            const int32_t* b = B + boff[(int64_t)j * nsub + s] + e;
            for (int64_t t = 0; t < nt; ++t) out[t] += b[t];
        }
    }
    free(B);
    free(boff);
    free(ext);
    free(d_fs);
    free(d_cs);
    free(d_cc);
    return 0;
}

/* Statistics of one row; returns 0 when var <= 0 (then S/N is 0). */
static int row_stats(const int32_t* y, int64_t T, int64_t* sum_out, double* inv_d) {
    int64_t sum = 0;
    for (int64_t t = 0; t < T; ++t) sum += y[t];
    const int64_t c = sum / T;   /* y >= 0: floor */
    int64_t q = 0;
    for (int64_t t = 0; t < T; ++t) q += ((int64_t)y[t] - c) * ((int64_t)y[t] - c);
    const int64_t r = sum - T * c;
    const double a = (double)q / (double)T;
    const double b = (double)r / (double)T;
    const double var = a - b * b;
    *sum_out = sum;
    if (var > 0.0) {
        *inv_d = 1.0 / (sqrt(var) * (double)T);
        return 1;
    }
    *inv_d = 0.0;
    return 0;
}

static double snr_of(int64_t T, int64_t S, int64_t w, int64_t sum, double inv_d) {
    const int64_t N = T * S - w * sum;
    return ((double)N * inv_d) * (1.0 / sqrt((double)w));
}

/* Widths increase (the callers sort them). */
int txo_boxcar_peaks(const int32_t* y, int ndm, int64_t nt, int64_t pitch, const int32_t* widths, int nw, double* snr,
                     int32_t* width, int64_t* time, int nthreads) {
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4)
    for (int d = 0; d < ndm; ++d) {
        const int32_t* row = y + (int64_t)d * pitch;
        int64_t sum = 0;
        double inv_d = 0.0;
        snr[d] = 0.0;
        width[d] = widths[0];
        time[d] = 0;
        if (!row_stats(row, nt, &sum, &inv_d)) continue;
        int64_t* P = malloc(sizeof(int64_t) * (size_t)(nt + 1));
        P[0] = 0;
        for (int64_t t = 0; t < nt; ++t) P[t + 1] = P[t] + row[t];
        int have = 0;
        for (int k = 0; k < nw; ++k) {
            const int64_t w = widths[k];
            if (w > nt) continue;
            int64_t bt = 0, bs = P[w] - P[0];
            for (int64_t t = 1; t + w <= nt; ++t)
                if (P[t + w] - P[t] > bs) {
                    bs = P[t + w] - P[t];
                    bt = t;
                }
            const double sn = snr_of(nt, bs, w, sum, inv_d);
            if (!have || sn > snr[d]) {
                snr[d] = sn;
                width[d] = (int32_t)w;
                time[d] = bt;
                have = 1;
            }
        }
        free(P);
    }
    return 0;
}

/* Thresholded points (d, t, best width, S/N) with S/N >= gamma, in (d, t)
 * order; returns the count (records beyond cap are counted, not stored). */
int64_t txo_candidates(const int32_t* y, int ndm, int64_t nt, int64_t pitch, const int32_t* widths, int nw,
                       double gamma, int32_t* cd, int64_t* ct, int32_t* cw, double* cs, int64_t cap, int nthreads) {
    int64_t* counts = calloc((size_t)ndm + 1, sizeof(int64_t));
    /* two passes: count per row, then write at the row's offset */
    for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4)
        for (int d = 0; d < ndm; ++d) {
            const int32_t* row = y + (int64_t)d * pitch;
            int64_t sum = 0;
            double inv_d = 0.0;
            if (!row_stats(row, nt, &sum, &inv_d)) continue;
            int64_t* P = malloc(sizeof(int64_t) * (size_t)(nt + 1));
            P[0] = 0;
            for (int64_t t = 0; t < nt; ++t) P[t + 1] = P[t] + row[t];
            int64_t k = pass ? counts[d] : 0;
            for (int64_t t = 0; t < nt; ++t) {
                double bs = 0.0;
                int bw = -1;
                for (int i = 0; i < nw; ++i) {
                    const int64_t w = widths[i];
                    if (t + w > nt) continue;
                    const double sn = snr_of(nt, P[t + w] - P[t], w, sum, inv_d);
                    if (bw < 0 || sn > bs) {
                        bs = sn;
                        bw = (int)w;
                    }
                }
                if (bw < 0 || !(bs >= gamma)) continue;
                if (pass && k < cap) {
                    cd[k] = d;
                    ct[k] = t;
                    cw[k] = bw;
                    cs[k] = bs;
                }
                ++k;
            }
            if (!pass) counts[d] = k;
            free(P);
        }
        if (!pass) { /* exclusive prefix over rows */
            int64_t run = 0;
            for (int d = 0; d < ndm; ++d) {
                const int64_t n = counts[d];
                counts[d] = run;
                run += n;
            }
            counts[ndm] = run;
        }
    }
    const int64_t total = counts[ndm];
    free(counts);
    return total;
}

int txo_max_threads(void) { return omp_get_max_threads(); }
