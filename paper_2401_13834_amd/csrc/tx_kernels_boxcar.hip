// Boxcar matched filter for gfx950 (MI355X): per-DM noise statistics, peak
// S/N over the boxcar widths, and the thresholded DM-time candidates.
#include "tx_internal.h"

#pragma clang fp contract(off)

namespace tx {

// ---------------------------------------------------------------------------
// Boxcar matched filter: one workgroup per DM row.
// Pass 1: exact sums of y and y^2 (uint64, exact for values < 2^21 and
// rows <= 2^20).  Then c = floor(sum/T), Q = sum y^2 - 2 c sum + T c^2
// (= sum (y - c)^2 exactly, evaluated mod 2^64), var, sigma, 1/(sigma T).
// For each width the least window sum S* whose S/N reaches gamma is found by
// bisection with the same float64 expression, so the per-window threshold
// test is an integer compare.
// Pass 2, per tile of 4096 window starts: the running sum P (uint32; window
// sums are exact as differences) of the tile plus the longest window in LDS,
// then every (start, width): track the largest sum per width (earliest start)
// and flag starts that pass a threshold; flagged starts compute the S/N of
// every width and append (row, t, best width, snr).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double snr_of(int64_t T, int64_t S, int64_t w, int64_t sum, double inv_d, double rsw) {
    const int64_t N = T * S - w * sum;
    return (static_cast<double>(N) * inv_d) * rsw;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int NWT>
__global__ __launch_bounds__(kThreads) void boxcar_kernel(BoxcarArgs a) {
    __shared__ uint32_t P[kBoxTile + TX_MAX_WIDTH + 8];
    __shared__ unsigned long long red1[kWaves], red2[kWaves];
    __shared__ int redbad[kWaves];
    __shared__ uint32_t scan_tot[kWaves];
    __shared__ int32_t sthr[TX_MAX_WIDTHS];
    __shared__ double sh_inv_d;
    __shared__ long long sh_sum;
    __shared__ int sh_state;                          // 0 ok, 1 zero variance, 2 out of range
    __shared__ int32_t wS[kWaves][NWT];
    __shared__ int32_t wT[kWaves][NWT];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int T = a.nt;

    for (int row = blockIdx.x; row < a.ndm; row += gridDim.x) {
        const int32_t* __restrict__ y = a.y + static_cast<size_t>(row) * a.pitch;
        // ---- pass 1: moments -------------------------------------------
        unsigned long long s1 = 0, s2 = 0;
        int bad = 0;
        for (int t = tid; t < T; t += kThreads) {
            const int32_t v = y[t];
            bad |= (v < 0) | (v >= TX_MAX_VALUE);
            const uint32_t u = static_cast<uint32_t>(v);
            s1 += u;
            s2 += static_cast<unsigned long long>(u) * u;
        }
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        bad = __any(bad) ? 1 : 0;
        if (lane == 0) {
            red1[wave] = s1;
            red2[wave] = s2;
            redbad[wave] = bad;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long S1 = 0, S2 = 0;
            int B = 0;
            for (int w = 0; w < kWaves; ++w) {
                S1 += red1[w];
                S2 += red2[w];
                B |= redbad[w];
            }
            int state = B ? 2 : 0;
            double inv_d = 0.0;
            const long long sum = static_cast<long long>(S1);
            if (!B) {
                const long long c = sum / T;
                const long long r = sum - static_cast<long long>(T) * c;
                const unsigned long long q = S2 - 2ull * static_cast<unsigned long long>(c) * S1 +
                                             static_cast<unsigned long long>(T) * static_cast<unsigned long long>(c) *
                                                 static_cast<unsigned long long>(c);
                const double av = static_cast<double>(q) / static_cast<double>(T);
                const double bv = static_cast<double>(r) / static_cast<double>(T);
                const double var = av - bv * bv;
                if (var > 0.0) {
                    const double sigma = __builtin_sqrt(var);
                    inv_d = 1.0 / (sigma * static_cast<double>(T));
                } else {
                    state = 1;
                }
            }
            sh_inv_d = inv_d;
            sh_sum = sum;
            sh_state = state;
        }
        __syncthreads();
        const int state = sh_state;
        const double inv_d = sh_inv_d;
        const long long sum = sh_sum;
        if (state != 0) {
            if (tid == 0 && a.want_peaks) {
                a.snr[row] = state == 1 ? 0.0 : __builtin_nan("");
                a.width[row] = state == 1 ? a.widths[0] : -1;
                a.time[row] = state == 1 ? 0 : -1;
            }
            __syncthreads();
            continue;
        }
        // Per-width threshold on the window sum (least S with snr >= gamma).
        if (a.want_cands && tid < a.nw) {
            const int64_t w = a.widths[tid];
            const double rsw = a.rsw[tid];
            int64_t lo = INT32_MIN, hi = INT32_MAX;
            int32_t res;
            if (snr_of(T, lo, w, sum, inv_d, rsw) >= a.gamma) {
                res = INT32_MIN;
            } else if (!(snr_of(T, hi, w, sum, inv_d, rsw) >= a.gamma)) {
                res = INT32_MAX;                      // never reached: window sums are < 2^31 - 1
            } else {
                while (hi - lo > 1) {                 // snr(lo) < gamma <= snr(hi)
                    const int64_t mid = lo + (hi - lo) / 2;
                    if (snr_of(T, mid, w, sum, inv_d, rsw) >= a.gamma) hi = mid; else lo = mid;
                }
                res = static_cast<int32_t>(hi);
            }
            sthr[tid] = res;
        }
        __syncthreads();

        // ---- pass 2: running sums and windows ----------------------------
        int32_t bestS[NWT];
        int32_t bestT[NWT];
#pragma unroll
        for (int k = 0; k < NWT; ++k) {
            bestS[k] = INT32_MIN;
            bestT[k] = 0;
        }
        const int L = kBoxTile + a.wmax;              // running-sum values needed past P[t0]
        uint32_t carry = 0;
        for (int t0 = 0; t0 < T; t0 += kBoxTile) {
            // inclusive scan of y[t0 .. t0 + L) (zeros past T) -> P[1 .. L]
            uint32_t run = carry;
            if (tid == 0) P[0] = carry;
            for (int k0 = 0; k0 < L; k0 += 4 * kThreads) {
                const int k = k0 + 4 * tid;
                uint32_t v0 = 0, v1 = 0, v2 = 0, v3 = 0;
                const int64_t t = static_cast<int64_t>(t0) + k;
                if (k < L) {
                    if (t + 0 < T) v0 = static_cast<uint32_t>(y[t + 0]);
                    if (t + 1 < T && k + 1 < L) v1 = static_cast<uint32_t>(y[t + 1]);
                    if (t + 2 < T && k + 2 < L) v2 = static_cast<uint32_t>(y[t + 2]);
                    if (t + 3 < T && k + 3 < L) v3 = static_cast<uint32_t>(y[t + 3]);
                }
                const uint32_t p1 = v0, p2 = p1 + v1, p3 = p2 + v2, p4 = p3 + v3;
                uint32_t incl = p4;                   // inclusive scan of thread totals in the wave
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t n = __shfl_up(incl, o);
                    if (lane >= o) incl += n;
                }
                if (lane == 63) scan_tot[wave] = incl;
                __syncthreads();
                uint32_t before = run;
                for (int w = 0; w < wave; ++w) before += scan_tot[w];
                const uint32_t excl = before + incl - p4;
                if (k < L) {
                    P[k + 1] = excl + p1;
                    if (k + 1 < L) P[k + 2] = excl + p2;
                    if (k + 2 < L) P[k + 3] = excl + p3;
                    if (k + 3 < L) P[k + 4] = excl + p4;
                }
                uint32_t round = 0;
                for (int w = 0; w < kWaves; ++w) round += scan_tot[w];
                run += round;
                __syncthreads();
            }
            // windows
            uint32_t Pt[kBoxPer];
#pragma unroll
            for (int r = 0; r < kBoxPer; ++r) Pt[r] = P[tid + kThreads * r];
            uint32_t flags = 0;
#pragma unroll
            for (int k = 0; k < NWT; ++k) {
                if (k < a.nw) {
                    const int w = a.widths[k];
                    if (w <= T) {
                        const int32_t thr = a.want_cands ? sthr[k] : INT32_MAX;
#pragma unroll
                        for (int r = 0; r < kBoxPer; ++r) {
                            const int t = t0 + tid + kThreads * r;
                            const bool valid = t + w <= T;
                            const int32_t S = static_cast<int32_t>(P[tid + kThreads * r + w] - Pt[r]);
                            if (valid && S > bestS[k]) {
                                bestS[k] = S;
                                bestT[k] = t;
                            }
                            if (valid && S >= thr) flags |= 1u << r;
                        }
                    }
                }
            }
            if (flags) {
                for (int r = 0; r < kBoxPer; ++r) {
                    if (!(flags & (1u << r))) continue;
                    const int t = t0 + tid + kThreads * r;
                    double bs = 0.0;
                    int bw = -1;
                    for (int k = 0; k < a.nw; ++k) {
                        const int w = a.widths[k];
                        if (w > T || t + w > T) continue;
                        const int32_t S = static_cast<int32_t>(P[tid + kThreads * r + w] - Pt[r]);
                        const double sn = snr_of(T, S, w, sum, inv_d, a.rsw[k]);
                        if (bw < 0 || sn > bs) {
                            bs = sn;
                            bw = w;
                        }
                    }
                    const unsigned long long idx = atomicAdd(a.count, 1ull);
                    if (static_cast<long long>(idx) < a.cap) {
                        tx_cand c;
                        c.dm_index = row;
                        c.width = bw;
                        c.time = t;
                        c.snr = bs;
                        a.cands[idx] = c;
                    }
                }
            }
            carry = P[kBoxTile];
            __syncthreads();
        }
        // ---- peak: reduce (largest S, earliest t) per width ------------------
        if (a.want_peaks) {
#pragma unroll
            for (int k = 0; k < NWT; ++k) {
                int32_t S = bestS[k];
                int32_t t = bestT[k];
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const int32_t S2 = __shfl_xor(S, o);
                    const int32_t t2 = __shfl_xor(t, o);
                    if (S2 > S || (S2 == S && t2 < t)) {
                        S = S2;
                        t = t2;
                    }
                }
                if (lane == 0) {
                    wS[wave][k] = S;
                    wT[wave][k] = t;
                }
            }
            __syncthreads();
            if (tid == 0) {
                double bs = 0.0;
                int bw = -1;
                long long bt = 0;
                for (int k = 0; k < a.nw; ++k) {
                    const int w = a.widths[k];
                    if (w > T) continue;
                    int32_t S = wS[0][k], t = wT[0][k];
                    for (int v = 1; v < kWaves; ++v)
                        if (wS[v][k] > S || (wS[v][k] == S && wT[v][k] < t)) {
                            S = wS[v][k];
                            t = wT[v][k];
                        }
                    const double sn = snr_of(T, S, w, sum, inv_d, a.rsw[k]);
                    if (bw < 0 || sn > bs) {
                        bs = sn;
                        bw = w;
                        bt = t;
                    }
                }
                if (bw < 0) {
                    bs = 0.0;
                    bw = a.widths[0];
                    bt = 0;
                }
                a.snr[row] = bs;
                a.width[row] = bw;
                a.time[row] = bt;
            }
        }
        __syncthreads();
    }
}

__global__ void zero_u64_kernel(unsigned long long* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

hipError_t launch_boxcar(const BoxcarArgs& a, hipStream_t stream) {
    if (a.want_cands) {
        hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, stream, a.count);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.ndm <= 0) return hipSuccess;
    const int grid = a.ndm;
    const int prof = prof_begin(TX_KERNEL_BOXCAR, stream);
    if (a.nw <= 8)
        hipLaunchKernelGGL(boxcar_kernel<8>, dim3(grid), dim3(kThreads), 0, stream, a);
    else if (a.nw <= 16)
        hipLaunchKernelGGL(boxcar_kernel<16>, dim3(grid), dim3(kThreads), 0, stream, a);
    else
        hipLaunchKernelGGL(boxcar_kernel<32>, dim3(grid), dim3(kThreads), 0, stream, a);
    const hipError_t e = hipGetLastError();
    prof_end(prof, stream);
    return e;
}

}  // namespace tx
