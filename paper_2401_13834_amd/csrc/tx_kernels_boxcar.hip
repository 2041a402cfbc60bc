// Boxcar matched filter for gfx950 (MI355X): per-DM noise statistics, peak
// S/N over the boxcar widths, and the thresholded DM-time candidates.
//
// One workgroup per DM row (the batch form walks the rows of many jobs with a
// persistent grid).  Per row:
//  1. exact sums of y and y^2 (uint64; exact for values < 2^21 and rows
//     <= 2^20), then c = floor(sum/T), Q = sum y^2 - 2 c sum + T c^2
//     (= sum (y - c)^2, evaluated mod 2^64), var = Q/T - (r/T)^2, sigma and
//     1/(sigma T) in float64;
//  2. per width, the least window sum S* whose S/N reaches gamma, by bisection
//     with the same float64 expression, so the per-window test is an integer
//     compare;
//  3. per tile of 4096 window starts: the tile's running sums (exclusive
//     prefix, uint32; window sums are exact as differences) of 4096 + the
//     longest width samples in LDS; every (start, width) updates the largest
//     sum per width (earliest start) and a per-start flag max(S - S*); flagged
//     starts compute the S/N of every width and append (row, t, best width,
//     snr) to the candidate list.
// Thread tid owns the starts t0 + 1024 k + 4 tid + r (k, r < 4), so its own
// running sums and those a window of width 4m needs are aligned 16-byte LDS
// reads.
#include <algorithm>

#include "tx_internal.h"

#pragma clang fp contract(off)

namespace tx {

template <int NWT>
struct BoxShared {
    __align__(16) uint32_t P[kBoxTile + TX_MAX_WIDTH + 16];
    unsigned long long red1[kWaves], red2[kWaves];
    int redbad[kWaves];
    uint32_t wtot[kWaves];
    int32_t sthr[TX_MAX_WIDTHS];
    int32_t wd[TX_MAX_WIDTHS];     // widths and 1/sqrt(width) of the row's job, for
    double rs[TX_MAX_WIDTHS];      // run-time indexing (no private copy of the arguments)
    double inv_d;
    long long sum;
    int state;
    int32_t wS[kWaves][NWT];
    int32_t wT[kWaves][NWT];
};

__device__ __forceinline__ double snr_of(int64_t T, int64_t S, int64_t w, int64_t sum, double inv_d, double rsw) {
    const int64_t N = T * S - w * sum;
    return (static_cast<double>(N) * inv_d) * rsw;
}

template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Exclusive running sums of y[t0 + e], e in [e0, e0 + 4096) (zeros past the
// row), written to P[e]; returns the round total.  Thread tid owns 16
// consecutive samples.
__device__ __forceinline__ uint32_t scan_round(const TX_GLOBAL int32_t* __restrict__ y, int T, int t0, int e0, int L,
                                               uint32_t base, uint32_t* P, uint32_t* wtot, bool vec, int tid) {
    const int lane = tid & 63, wave = tid >> 6;
    const int e = e0 + 16 * tid;
    uint32_t v[16];
    const int64_t t = static_cast<int64_t>(t0) + e;
    if (vec && e + 16 <= L && t + 16 <= T) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint4 q = *reinterpret_cast<const TX_GLOBAL uint4*>(y + t + 4 * k);
            v[4 * k] = q.x;
            v[4 * k + 1] = q.y;
            v[4 * k + 2] = q.z;
            v[4 * k + 3] = q.w;
        }
    } else {
        // Valid samples of this lane in this round (the count changes with the
        // tile, so no per-element condition is hoisted out of the tile loop).
        const int64_t lim = min(static_cast<int64_t>(L - e), static_cast<int64_t>(T) - t);
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = k < lim ? static_cast<uint32_t>(y[t + k]) : 0u;
    }
    uint32_t ex[16];
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        ex[k] = run;
        run += v[k];
    }
    uint32_t incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t n = __shfl_up(incl, o);
        if (lane >= o) incl += n;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    uint32_t before = base;
    for (int w = 0; w < wave; ++w) before += wtot[w];
    before += incl - run;
    if (e < L) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            *reinterpret_cast<uint4*>(P + e + 4 * k) =
                make_uint4(before + ex[4 * k], before + ex[4 * k + 1], before + ex[4 * k + 2], before + ex[4 * k + 3]);
    }
    const uint32_t total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
    __syncthreads();
    return total;
}

// One tile of 4096 window starts.  TAIL: some windows reach past the row end.
// Wavefront max / min of an int32 with DPP moves (quad, half-row and row
// permutes, then the row broadcasts of 15 and 31); the result is read from
// lane 63.
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));  // row_mirror
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x142, 0xA, 0xF, false));  // row_bcast15
    v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x143, 0xC, 0xF, false));  // row_bcast31
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x142, 0xA, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x143, 0xC, 0xF, false));
    return __builtin_amdgcn_readlane(v, 63);
}

// One tile of 4096 window starts.  TAIL: some windows reach past the row end.
// Per width slot, each lane keeps only the largest sum of its 16 starts; the
// wavefront's largest sum is compared with the wavefront's best so far
// (kept in LDS per wavefront) and only when it beats it (a few tiles per
// row) does the wavefront look up the earliest start reaching it.  Candidate
// flags take max(S - S*) over pairs of width slots with one 3-input max.
// Width slots past the row's widths repeat its last width, so the loop has no
// per-width branches.
template <int NWT, bool TAIL, bool CANDS>
__device__ __forceinline__ void boxcar_tile(const BoxcarArgs& a, BoxShared<NWT>& sh, int row, int t0, long long sum,
                                            double inv_d, int tid) {
    const int wave = tid >> 6;
    const int T = a.nt;
    const int lb = 4 * tid;     // this lane's first start in the tile
    uint32_t Pt[4][4];
    int32_t mx[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint4 q = *reinterpret_cast<const uint4*>(sh.P + lb + 1024 * k);
        Pt[k][0] = q.x;
        Pt[k][1] = q.y;
        Pt[k][2] = q.z;
        Pt[k][3] = q.w;
#pragma unroll
        for (int r = 0; r < 4; ++r) mx[k][r] = INT32_MIN;
    }
#pragma unroll 1
    for (int i = 0; i < NWT; i += 2) {
        // Per-width values come from LDS, which keeps the registers free.
        const int w0 = sh.wd[i], w1 = sh.wd[i + 1];
        const int32_t thr0 = CANDS ? max(sh.sthr[i], 0) : 0;
        const int32_t thr1 = CANDS ? max(sh.sthr[i + 1], 0) : 0;
        int32_t tm0 = INT32_MIN, tm1 = INT32_MIN;
        const uint32_t* p0 = sh.P + lb + w0;
        const uint32_t* p1 = sh.P + lb + w1;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int base = 1024 * k + 4 * tid;
            const uint2 u0 = *reinterpret_cast<const uint2*>(p0 + 1024 * k);
            const uint2 u1 = *reinterpret_cast<const uint2*>(p0 + 1024 * k + 2);
            const uint2 v0 = *reinterpret_cast<const uint2*>(p1 + 1024 * k);
            const uint2 v1 = *reinterpret_cast<const uint2*>(p1 + 1024 * k + 2);
            const uint32_t A[4] = {u0.x, u0.y, u1.x, u1.y};
            const uint32_t B[4] = {v0.x, v0.y, v1.x, v1.y};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int32_t S0 = static_cast<int32_t>(A[r] - Pt[k][r]);
                const int32_t S1 = static_cast<int32_t>(B[r] - Pt[k][r]);
                const int t = t0 + base + r;
                const bool ok0 = !TAIL || t + w0 <= T;   // no window past the row end
                const bool ok1 = !TAIL || t + w1 <= T;
                tm0 = max(tm0, ok0 ? S0 : INT32_MIN);
                tm1 = max(tm1, ok1 ? S1 : INT32_MIN);
                if (CANDS) {
                    // valid sums are >= 0 and thresholds in [0, 2^31), so S - thr cannot wrap
                    const int32_t d0 = ok0 ? S0 - thr0 : -1;
                    const int32_t d1 = ok1 ? S1 - thr1 : -1;
                    mx[k][r] = max(max(mx[k][r], d0), d1);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ii = i + h;
            const int w = h ? w1 : w0;
            const int32_t wm = wave_max_i32(h ? tm1 : tm0);
            if (wm > sh.wS[wave][ii]) {                 // wavefront-uniform, a few tiles per row
                int32_t first = INT32_MAX;
#pragma unroll 1
                for (int kr = 15; kr >= 0; --kr) {      // rolled: this path is rare
                    const int e = 1024 * (kr >> 2) + 4 * tid + (kr & 3);
                    const int t = t0 + e;
                    const int32_t S = static_cast<int32_t>(sh.P[e + w] - sh.P[e]);
                    const bool ok = !TAIL || t + w <= T;
                    first = (ok && S == wm) ? t : first;
                }
                const int32_t ft = wave_min_i32(first);
                if ((tid & 63) == 0) {
                    sh.wS[wave][ii] = wm;
                    sh.wT[wave][ii] = ft;
                }
            }
        }
        // Keep each width pair's LDS reads next to their arithmetic (the
        // scheduler would otherwise hoist every width's reads and run out of
        // registers).
        __builtin_amdgcn_sched_barrier(0);
    }
    if (CANDS) {
        // Flagged starts (rare) as a bit mask, then one start at a time.
        uint32_t flags = 0;
#pragma unroll
        for (int k = 3; k >= 0; --k)
#pragma unroll
            for (int r = 3; r >= 0; --r) flags = (flags << 1) | (mx[k][r] >= 0 ? 1u : 0u);   // bit 4k + r
        while (flags) {
            const int kr = __builtin_ctz(flags);
            flags &= flags - 1;
            const int e = 1024 * (kr >> 2) + 4 * tid + (kr & 3);
            const int t = t0 + e;
            const uint32_t pt = sh.P[e];
            double bs = 0.0;
            int bw = -1;
            for (int i = 0; i < a.ne; ++i) {
                const int w = sh.wd[i];
                if (t + w > T) continue;
                const int32_t S = static_cast<int32_t>(sh.P[e + w] - pt);
                const double sn = snr_of(T, S, w, sum, inv_d, sh.rs[i]);
                if (bw < 0 || sn > bs) {
                    bs = sn;
                    bw = w;
                }
            }
            {
                const unsigned long long slot = atomicAdd(a.count, 1ull);
                if (static_cast<long long>(slot) < a.cap) {
                    tx_cand c;
                    c.dm_index = row;
                    c.width = bw;
                    c.time = t;
                    c.snr = bs;
                    to_global(a.cands)[slot] = c;
                }
            }
        }
    }
}

template <int NWT>
__device__ __forceinline__ void boxcar_row(const BoxcarArgs& a, int row, BoxShared<NWT>& sh) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int T = a.nt;
    const TX_GLOBAL int32_t* __restrict__ y = to_global(a.y) + static_cast<size_t>(row) * a.pitch;
    const bool vec = ((reinterpret_cast<uintptr_t>(a.y) + static_cast<uintptr_t>(row) * a.pitch * 4) & 15) == 0;
    if (tid < NWT) {
        int32_t w = 0;
        double r = 0.0;
#pragma unroll
        for (int k = 0; k < NWT; ++k)          // compile-time indices only
            if (k == tid) {
                w = a.widths[k];
                r = a.rsw[k];
            }
        sh.wd[tid] = w;
        sh.rs[tid] = r;
    }

    // ---- moments ----------------------------------------------------------
    unsigned long long s1 = 0, s2 = 0;
    int bad = 0;
    const int nvec = vec ? T / 4 : 0;
    for (int v = tid; v < nvec; v += kThreads) {
        const int4 q = *reinterpret_cast<const TX_GLOBAL int4*>(y + 4 * v);
        const int32_t e[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            bad |= (e[k] < 0) | (e[k] >= TX_MAX_VALUE);
            const uint32_t u = static_cast<uint32_t>(e[k]);
            s1 += u;
            s2 += static_cast<unsigned long long>(u) * u;
        }
    }
    for (int t = 4 * nvec + tid; t < T; t += kThreads) {
        const int32_t e = y[t];
        bad |= (e < 0) | (e >= TX_MAX_VALUE);
        const uint32_t u = static_cast<uint32_t>(e);
        s1 += u;
        s2 += static_cast<unsigned long long>(u) * u;
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    bad = __any(bad) ? 1 : 0;
    if (lane == 0) {
        sh.red1[wave] = s1;
        sh.red2[wave] = s2;
        sh.redbad[wave] = bad;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long S1 = 0, S2 = 0;
        int B = 0;
        for (int w = 0; w < kWaves; ++w) {
            S1 += sh.red1[w];
            S2 += sh.red2[w];
            B |= sh.redbad[w];
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
        sh.inv_d = inv_d;
        sh.sum = sum;
        sh.state = state;
    }
    __syncthreads();
    const int state = sh.state;
    const double inv_d = sh.inv_d;
    const long long sum = sh.sum;
    if (state != 0) {
        if (tid == 0 && a.want_peaks) {
            to_global(a.snr)[row] = state == 1 ? 0.0 : __builtin_nan("");
            to_global(a.width)[row] = state == 1 ? a.w_first : -1;
            to_global(a.time)[row] = state == 1 ? 0 : -1;
        }
        __syncthreads();
        return;
    }
    // ---- per-width thresholds ------------------------------------------------
    if (a.want_cands && tid < NWT) {
        const int64_t w = sh.wd[tid];
        const double rsw = sh.rs[tid];
        int64_t lo = INT32_MIN, hi = INT32_MAX;
        int32_t res;
        if (snr_of(T, lo, w, sum, inv_d, rsw) >= a.gamma) {
            res = INT32_MIN;
        } else if (!(snr_of(T, hi, w, sum, inv_d, rsw) >= a.gamma)) {
            res = INT32_MAX;                          // never reached: window sums are < 2^31 - 1
        } else {
            while (hi - lo > 1) {                     // snr(lo) < gamma <= snr(hi)
                const int64_t mid = lo + (hi - lo) / 2;
                if (snr_of(T, mid, w, sum, inv_d, rsw) >= a.gamma) hi = mid; else lo = mid;
            }
            res = static_cast<int32_t>(hi);
        }
        sh.sthr[tid] = res;
    }
    __syncthreads();

    // ---- tiles ------------------------------------------------------------------
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NWT; ++i) {
            sh.wS[wave][i] = INT32_MIN;   // this wavefront's best sum per width so far
            sh.wT[wave][i] = 0;
        }
    }
    const int L = kBoxTile + a.wmax;
    for (int t0 = 0; a.ne > 0 && t0 < T; t0 += kBoxTile) {
        // The thread index, made opaque to the compiler in every tile: else it
        // hoists dozens of lane-dependent masks and addresses out of this loop
        // and spills them.
        int tv = tid;
        asm volatile("" : "+v"(tv));
        const uint32_t tot = scan_round(y, T, t0, 0, L, 0u, sh.P, sh.wtot, vec, tv);
        uint32_t tot2 = 0;
        if (L > kBoxTile) tot2 = scan_round(y, T, t0, kBoxTile, L, tot, sh.P, sh.wtot, vec, tv);
        if (tid == 0) sh.P[L] = tot + tot2;
        __syncthreads();
        const bool tail = t0 + kBoxTile + a.wmax > T;
        if (a.want_cands) {
            if (tail) boxcar_tile<NWT, true, true>(a, sh, row, t0, sum, inv_d, tv);
            else boxcar_tile<NWT, false, true>(a, sh, row, t0, sum, inv_d, tv);
        } else {
            if (tail) boxcar_tile<NWT, true, false>(a, sh, row, t0, sum, inv_d, tv);
            else boxcar_tile<NWT, false, false>(a, sh, row, t0, sum, inv_d, tv);
        }
        __syncthreads();
    }
    // ---- peak: reduce (largest S, earliest t) per width ---------------------------
    if (a.want_peaks) {
        __syncthreads();
        if (tid == 0) {
            double bs = 0.0;
            int bw = -1;
            long long bt = 0;
            for (int i = 0; i < a.ne; ++i) {
                const int w = sh.wd[i];
                int32_t S = sh.wS[0][i], t = sh.wT[0][i];
                for (int v = 1; v < kWaves; ++v)
                    if (sh.wS[v][i] > S || (sh.wS[v][i] == S && sh.wT[v][i] < t)) {
                        S = sh.wS[v][i];
                        t = sh.wT[v][i];
                    }
                const double sn = snr_of(T, S, w, sum, inv_d, sh.rs[i]);
                if (bw < 0 || sn > bs) {
                    bs = sn;
                    bw = w;
                    bt = t;
                }
            }
            if (bw < 0) {
                bs = 0.0;
                bw = a.w_first;
                bt = 0;
            }
            to_global(a.snr)[row] = bs;
            to_global(a.width)[row] = bw;
            to_global(a.time)[row] = bt;
        }
    }
    __syncthreads();
}

template <int NWT>
__global__ __launch_bounds__(kThreads) void boxcar_kernel(BoxcarArgs a) {
    __shared__ BoxShared<NWT> sh;
    const int row = static_cast<int>(blockIdx.x);        // grid = rows
    if (row < a.ndm) boxcar_row<NWT>(a, row, sh);
}

__device__ __forceinline__ int find_row_job(const int* __restrict__ prefix, int njobs, int v) {
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// Batch form: one workgroup per row of all jobs (job of a row by prefix sums);
// the grid may exceed the batch's rows (a captured graph is sized for the
// largest batch) and workgroups past the last row exit at once.
template <int NWT>
__global__ __launch_bounds__(kThreads) void boxcar_batch_kernel(const BoxcarArgs* __restrict__ jobs,
                                                                const int* __restrict__ prefix,
                                                                const int* __restrict__ njobs_p) {
    __shared__ BoxShared<NWT> sh;
    const int njobs = *njobs_p;
    const int total = prefix[njobs];
    const int v = static_cast<int>(blockIdx.x);
    if (v >= total) return;
    const int jb = find_row_job(prefix, njobs, v);
    boxcar_row<NWT>(jobs[jb], v - prefix[jb], sh);
}

__global__ void zero_u64_kernel(unsigned long long* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

__global__ void zero_counts_kernel(const BoxcarArgs* __restrict__ jobs, const int* __restrict__ njobs_p) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < *njobs_p && jobs[j].want_cands) *jobs[j].count = 0ull;
}

// ---------------------------------------------------------------------------
// Launches.
// ---------------------------------------------------------------------------
hipError_t launch_boxcar(const BoxcarArgs& a, hipStream_t stream) {
    if (a.want_cands) {
        hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, stream, a.count);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.ndm <= 0) return hipSuccess;
    const int grid = a.ndm;
    const int prof = prof_begin(TX_KERNEL_BOXCAR, stream);
    switch (boxcar_nwt(a.ne)) {
        case 4: hipLaunchKernelGGL(boxcar_kernel<4>, dim3(grid), dim3(kThreads), 0, stream, a); break;
        case 8: hipLaunchKernelGGL(boxcar_kernel<8>, dim3(grid), dim3(kThreads), 0, stream, a); break;
        case 12: hipLaunchKernelGGL(boxcar_kernel<12>, dim3(grid), dim3(kThreads), 0, stream, a); break;
        case 16: hipLaunchKernelGGL(boxcar_kernel<16>, dim3(grid), dim3(kThreads), 0, stream, a); break;
        default: hipLaunchKernelGGL(boxcar_kernel<32>, dim3(grid), dim3(kThreads), 0, stream, a); break;
    }
    const hipError_t e = hipGetLastError();
    prof_end(prof, stream);
    return e;
}


hipError_t launch_boxcar_batch(int nwt, const BoxcarArgs* d_jobs, const int* d_prefix, const int* d_njobs, int grid,
                               hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    const int prof = prof_begin(TX_KERNEL_BOXCAR, stream);
    switch (boxcar_nwt(nwt)) {
        case 4: hipLaunchKernelGGL(boxcar_batch_kernel<4>, dim3(grid), dim3(kThreads), 0, stream, d_jobs, d_prefix, d_njobs); break;
        case 8: hipLaunchKernelGGL(boxcar_batch_kernel<8>, dim3(grid), dim3(kThreads), 0, stream, d_jobs, d_prefix, d_njobs); break;
        case 12: hipLaunchKernelGGL(boxcar_batch_kernel<12>, dim3(grid), dim3(kThreads), 0, stream, d_jobs, d_prefix, d_njobs); break;
        case 16: hipLaunchKernelGGL(boxcar_batch_kernel<16>, dim3(grid), dim3(kThreads), 0, stream, d_jobs, d_prefix, d_njobs); break;
        default: hipLaunchKernelGGL(boxcar_batch_kernel<32>, dim3(grid), dim3(kThreads), 0, stream, d_jobs, d_prefix, d_njobs); break;
    }
    const hipError_t e = hipGetLastError();
    prof_end(prof, stream);
    return e;
}

hipError_t launch_zero_counts(const BoxcarArgs* d_jobs, const int* d_njobs, int max_jobs, hipStream_t stream) {
    if (max_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_counts_kernel, dim3((max_jobs + 255) / 256), dim3(256), 0, stream, d_jobs, d_njobs);
    return hipGetLastError();
}

}  // namespace tx
