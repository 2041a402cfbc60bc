// Boxcar matched filter for gfx950 (MI355X): per-DM noise statistics, peak
// S/N over the boxcar widths, and the thresholded DM-time candidates
// (Sec. 2.4, Eq. 5; Sec. 2.5).
//
// One workgroup per DM row (the batch form takes the rows of many jobs).  The
// row is read from HBM once, in tiles of 4096 window starts:
//  * each tile's running sums (exclusive prefix, uint32: window sums are exact
//    as differences) of its 4096 + longest-width samples go to LDS; the same
//    loads accumulate the exact moments sum y and sum y^2 (uint64);
//  * per width, every lane keeps the largest window sum of its 16 starts; the
//    wavefront's largest is compared with the wavefront's best so far, and
//    only when it beats it (a few tiles per row) does the wavefront look up
//    the earliest start reaching it; the workgroup's largest sum per (tile,
//    width) is kept in LDS.
// Then c = floor(sum/T), Q = sum y^2 - 2 c sum + T c^2 (= sum (y - c)^2, mod
// 2^64), var = Q/T - (r/T)^2, sigma and 1/(sigma T) in float64 give the peak
// S/N, and per width the least window sum S* whose S/N reaches gamma
// (bisection with the same float64 expression).  Only tiles where some width's
// largest sum reaches its S* are read again to list candidates: a start is a
// candidate when some width passes, and is reported with the width of highest
// S/N.  Thread tid owns the starts t0 + tid + 256 j (j < 16).
#include <algorithm>

#include "tx_internal.h"

#pragma clang fp contract(off)

namespace tx {

// Largest dynamic LDS for the per-(tile, width) maxima; rows needing more
// read every tile again for candidates.
constexpr int kTileMaxLds = 16 * 1024;

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
    int32_t wS[kWaves][NWT];       // per wavefront: best sum per width so far, and
    int32_t wT[kWaves][NWT];       // its earliest start
};

extern __shared__ int32_t tx_box_tmax[];   // [tiles][NWT]: workgroup's largest sum per tile and width

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

// Wavefront max / min of an int32 with DPP (quad, half-row and row permutes,
// then the row broadcasts of 15 and 31); the result is read from lane 63.
// The moves' fallback value is the operation's identity, so each step
// compiles to one v_max/v_min with a DPP source instead of a move and an op
// (rows a broadcast does not write keep their value either way).
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x140, 0xF, 0xF, false));  // row_mirror
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x142, 0xA, 0xF, false));  // row_bcast15
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x143, 0xC, 0xF, false));  // row_bcast31
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0xB1, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x4E, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x141, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x140, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x142, 0xA, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x143, 0xC, 0xF, false));
    return __builtin_amdgcn_readlane(v, 63);
}

// Inclusive prefix sum over the wavefront's lanes with DPP: shifts of 1, 2,
// 4 and 8 lanes within each row of 16 (lanes without a source add the
// identity 0), then the row broadcasts of lanes 15 and 31 into the rows
// above them.  Each step is one v_add with a DPP source; no LDS traffic.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
    x += __builtin_amdgcn_update_dpp(0u, x, 0x111, 0xF, 0xF, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0u, x, 0x112, 0xF, 0xF, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0u, x, 0x114, 0xF, 0xF, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0u, x, 0x118, 0xF, 0xF, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0u, x, 0x142, 0xA, 0xF, false);   // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0u, x, 0x143, 0xC, 0xF, false);   // row_bcast:31 into rows 2, 3
    return x;
}

// Moments of the samples a thread loaded (exact; a value >= 2^21 or < 0 flags
// the row).
struct Moments {
    unsigned long long s1 = 0, s2 = 0;
    uint32_t bad = 0;
};

// Exclusive running sums of y[t0 + e] for e < L = 4096 + longest width
// (<= 5120; zeros past the row) into P[e], and P[L] = their total.  Thread
// tid owns the 20 consecutive samples from e = 20 tid.  COUNT: add the
// samples with e < 4096 (the tile's own) to the moments.
template <bool COUNT>
__device__ __forceinline__ void scan_tile(const TX_GLOBAL int32_t* __restrict__ y, int T, int t0, int L, uint32_t* P,
                                          uint32_t* wtot, bool vec, int tid, Moments& m) {
    constexpr int kPer = 20;
    const int lane = tid & 63, wave = tid >> 6;
    const int e = kPer * tid;
    uint32_t v[kPer];
    const int64_t t = static_cast<int64_t>(t0) + e;
    if (vec && e + kPer <= L && t + kPer <= T) {
#pragma unroll
        for (int k = 0; k < kPer / 4; ++k) {
            const uint4 q = *reinterpret_cast<const TX_GLOBAL uint4*>(y + t + 4 * k);
            v[4 * k] = q.x;
            v[4 * k + 1] = q.y;
            v[4 * k + 2] = q.z;
            v[4 * k + 3] = q.w;
        }
    } else {
        // Valid samples of this lane (the count changes with the tile, so no
        // per-element condition is hoisted out of the tile loop).
        const int64_t lim = min(static_cast<int64_t>(L - e), static_cast<int64_t>(T) - t);
#pragma unroll
        for (int k = 0; k < kPer; ++k) v[k] = k < lim ? static_cast<uint32_t>(y[t + k]) : 0u;
    }
    if (COUNT) {
        // The sums are used only when every sample is in [0, TX_MAX_VALUE)
        // (then ps < 20 * 2^21 and y^2 < 2^42: no wrap), so out-of-range
        // samples need only the flag, taken from the running maximum (as
        // unsigned, a negative sample is out of range too).
        constexpr uint32_t kMask = static_cast<uint32_t>(TX_MAX_VALUE) - 1u;
        const int own = min(kPer, kBoxTile - e);       // samples of this tile (the rest belong to the next)
        uint32_t ps = 0, mx = 0;
        if (own == kPer) {                             // all but the threads at the tile's end
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                mx = max(mx, v[k]);
                ps += v[k];
                m.s2 += static_cast<unsigned long long>(v[k]) * v[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const uint32_t x = k < own ? v[k] : 0u;
                mx = max(mx, x);
                ps += x;
                m.s2 += static_cast<unsigned long long>(x) * x;
            }
        }
        m.bad |= mx > kMask ? 1u : 0u;
        m.s1 += ps;
    }
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) run += v[k];
    const uint32_t incl = wave_incl_sum(run);
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wtot[w];
    before += incl - run;
    if (e < L) {
#pragma unroll
        for (int k = 0; k < kPer / 4; ++k) {
            const uint32_t p0 = before, p1 = p0 + v[4 * k], p2 = p1 + v[4 * k + 1], p3 = p2 + v[4 * k + 2];
            before = p3 + v[4 * k + 3];
            *reinterpret_cast<uint4*>(P + e + 4 * k) = make_uint4(p0, p1, p2, p3);
        }
    }
    if (tid == 0) P[L] = wtot[0] + wtot[1] + wtot[2] + wtot[3];
    __syncthreads();
}

// Peak search over one tile.  Lane tid owns the starts t0 + tid + 256 j
// (j < 16), so a wavefront reads 64 consecutive LDS words per load (no bank
// conflicts for any width).  TAIL: some windows reach past the row end.  Width
// slots past the row's widths repeat its last width.
template <int NWT, bool TAIL>
__device__ __forceinline__ void peak_tile(const BoxcarArgs& a, BoxShared<NWT>& sh, int tile, int t0, int tid,
                                          bool keep_tmax) {
    const int wave = tid >> 6;
    const int T = a.nt;
    uint32_t Pt[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) Pt[j] = sh.P[tid + 256 * j];
    int32_t tm[NWT];
#pragma unroll
    for (int i = 0; i < NWT; i += 2) {
        // Per-width values come from LDS, which keeps the registers free.
        const int w0 = sh.wd[i], w1 = sh.wd[i + 1];
        const uint32_t* p0 = sh.P + tid + w0;
        const uint32_t* p1 = sh.P + tid + w1;
        int32_t tm0 = INT32_MIN, tm1 = INT32_MIN;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int32_t S0 = static_cast<int32_t>(p0[256 * j] - Pt[j]);
            const int32_t S1 = static_cast<int32_t>(p1[256 * j] - Pt[j]);
            const int t = t0 + tid + 256 * j;
            tm0 = max(tm0, (!TAIL || t + w0 <= T) ? S0 : INT32_MIN);   // no window past the row end
            tm1 = max(tm1, (!TAIL || t + w1 <= T) ? S1 : INT32_MIN);
        }
        tm[i] = tm0;
        tm[i + 1] = tm1;
        // Keep each width pair's LDS reads next to their arithmetic.
        __builtin_amdgcn_sched_barrier(0);
    }
    // Wavefront maxima of all widths (independent reductions, interleaved).
    int32_t wm[NWT];
#pragma unroll
    for (int i = 0; i < NWT; ++i) wm[i] = wave_max_i32(tm[i]);
#pragma unroll 1
    for (int ii = 0; ii < NWT; ++ii) {
        // wm[ii] with a run-time ii: select among the (uniform) values.
        int32_t m = wm[0];
#pragma unroll
        for (int k = 1; k < NWT; ++k) m = (k == ii) ? wm[k] : m;
        if (keep_tmax && (tid & 63) == 0) atomicMax(&tx_box_tmax[tile * NWT + ii], m);
        if (m > sh.wS[wave][ii]) {                      // wavefront-uniform, a few tiles per row
            const int w = sh.wd[ii];
            int32_t first = INT32_MAX;
#pragma unroll 1
            for (int j = 15; j >= 0; --j) {             // rolled: this path is rare
                const int e = tid + 256 * j;
                const int t = t0 + e;
                const int32_t S = static_cast<int32_t>(sh.P[e + w] - sh.P[e]);
                first = ((!TAIL || t + w <= T) && S == m) ? t : first;
            }
            const int32_t ft = wave_min_i32(first);
            if ((tid & 63) == 0) {
                sh.wS[wave][ii] = m;
                sh.wT[wave][ii] = ft;
            }
        }
    }
}

// Candidates of one tile (rare: only tiles where some width's largest sum
// reaches its threshold S*).  Widths increase, so a strict ">" keeps the
// smaller width on equal S/N.
template <int NWT>
__device__ __forceinline__ void cand_tile(const BoxcarArgs& a, BoxShared<NWT>& sh, int row, int t0, long long sum,
                                          double inv_d, int tid) {
    const int T = a.nt;
#pragma unroll 1
    for (int j = 0; j < 16; ++j) {
        const int e = tid + 256 * j;
        const int t = t0 + e;
        const uint32_t pt = sh.P[e];
        bool pass = false;
        double bs = 0.0;
        int bw = -1;
        for (int i = 0; i < a.ne; ++i) {
            const int w = sh.wd[i];
            if (t + w > T) continue;
            const int32_t S = static_cast<int32_t>(sh.P[e + w] - pt);
            pass = pass || S >= max(sh.sthr[i], 0);       // window sums are >= 0
            const double sn = snr_of(T, S, w, sum, inv_d, sh.rs[i]);
            if (bw < 0 || sn > bs) {
                bs = sn;
                bw = w;
            }
        }
        if (!pass) continue;
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

// Widths and 1/sqrt(w) of the row's job into LDS, the wavefronts' per-width
// best cleared, and the per-(tile, width) maxima table reset.
template <int NWT>
__device__ __forceinline__ void row_setup(const BoxcarArgs& a, int ntiles, bool keep_tmax, BoxShared<NWT>& sh,
                                          int tid) {
    const int lane = tid & 63;
    const int wave = tid >> 6;
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
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NWT; ++i) {
            sh.wS[wave][i] = INT32_MIN;
            sh.wT[wave][i] = 0;
        }
    }
    if (keep_tmax)
        for (int k = tid; k < ntiles * NWT; k += kThreads) tx_box_tmax[k] = INT32_MIN;
    __syncthreads();
}

// Tiles [tlo, thi) of a row: running sums, exact moments (wavefront sums left
// in sh.red*), per-width best of every wavefront (sh.wS / sh.wT) and the
// per-(tile, width) maxima.
template <int NWT>
__device__ __forceinline__ void row_scan(const BoxcarArgs& a, int tlo, int thi, bool keep_tmax,
                                         const TX_GLOBAL int32_t* __restrict__ y, bool vec, BoxShared<NWT>& sh,
                                         int tid) {
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int T = a.nt;
    const int L = kBoxTile + a.wmax;
    Moments m;
    for (int tile = tlo; tile < thi; ++tile) {
        const int t0 = tile * kBoxTile;
        // The thread index, made opaque to the compiler in every tile: else it
        // hoists dozens of lane-dependent masks and addresses out of this loop
        // and spills them.
        int tv = tid;
        asm volatile("" : "+v"(tv));
        scan_tile<true>(y, T, t0, L, sh.P, sh.wtot, vec, tv, m);
        if (a.ne > 0) {
            if (t0 + kBoxTile + a.wmax > T) peak_tile<NWT, true>(a, sh, tile, t0, tv, keep_tmax);
            else peak_tile<NWT, false>(a, sh, tile, t0, tv, keep_tmax);
        }
        __syncthreads();
    }
    const unsigned long long s1 = wave_sum(m.s1);
    const unsigned long long s2 = wave_sum(m.s2);
    const int bad = __any(m.bad != 0) ? 1 : 0;
    if (lane == 0) {
        sh.red1[wave] = s1;
        sh.red2[wave] = s2;
        sh.redbad[wave] = bad;
    }
    __syncthreads();
}

// Statistics, the row's peak and (when asked) its candidates, from the state
// row_scan left in LDS.
template <int NWT>
__device__ __forceinline__ void row_finish(const BoxcarArgs& a, int row, int ntiles, bool keep_tmax,
                                           const TX_GLOBAL int32_t* __restrict__ y, bool vec, BoxShared<NWT>& sh,
                                           int tid) {
    const int T = a.nt;
    const int L = kBoxTile + a.wmax;
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

    // ---- peak: (largest S, earliest t) per width, then the best width -------------
    if (a.want_peaks && tid == 0) {
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

    // ---- candidates ------------------------------------------------------------------
    if (a.want_cands && a.ne > 0) {
        if (tid < a.ne) {
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
        for (int tile = 0; tile < ntiles; ++tile) {
            bool hit = !keep_tmax;
            if (keep_tmax)
                for (int i = 0; i < a.ne; ++i) hit = hit || tx_box_tmax[tile * NWT + i] >= max(sh.sthr[i], 0);
            if (!hit) continue;                           // workgroup-uniform
            Moments unused;
            scan_tile<false>(y, T, tile * kBoxTile, L, sh.P, sh.wtot, vec, tid, unused);
            cand_tile<NWT>(a, sh, row, tile * kBoxTile, sum, inv_d, tid);
            __syncthreads();
        }
    }
    __syncthreads();
}


template <int NWT>
__device__ __forceinline__ void boxcar_row(const BoxcarArgs& a, int row, BoxShared<NWT>& sh, int tid) {
    const TX_GLOBAL int32_t* __restrict__ y = to_global(a.y) + static_cast<size_t>(row) * a.pitch;
    const bool vec = ((reinterpret_cast<uintptr_t>(a.y) + static_cast<uintptr_t>(row) * a.pitch * 4) & 15) == 0;
    const int ntiles = (a.nt + kBoxTile - 1) / kBoxTile;
    const bool keep_tmax = a.tmax_ok != 0;
    row_setup<NWT>(a, ntiles, keep_tmax, sh, tid);
    row_scan<NWT>(a, 0, ntiles, keep_tmax, y, vec, sh, tid);
    row_finish<NWT>(a, row, ntiles, keep_tmax, y, vec, sh, tid);
}

// Single job: one workgroup per row.
template <int NWT>
// At least 5 waves per SIMD (at most 102 VGPRs).  When the kernel needed 113
// VGPRs (4 waves) the cap made it 7% faster despite a 3-dword spill; the
// current form needs 69 VGPRs with the cap (75 without) and spills nothing.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5))) void boxcar_kernel(BoxcarArgs a) {
    __shared__ BoxShared<NWT> sh;
    const int row = static_cast<int>(blockIdx.x);        // grid = rows
    if (row < a.ndm) boxcar_row<NWT>(a, row, sh, static_cast<int>(threadIdx.x));
}

__device__ __forceinline__ int find_row_job(const int* __restrict__ prefix, int njobs, int v) {
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// Batch form: persistent workgroups taking rows of all jobs (job of a row by
// prefix sums) from the launch's work counters.
template <int NWT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5))) void boxcar_batch_kernel(const BoxcarArgs* __restrict__ jobs,
                                                                const int* __restrict__ prefix_base,
                                                                const int* __restrict__ info, uint32_t* queue) {
    __shared__ BoxShared<NWT> sh;
    const int njobs = info[0];
    if (njobs <= 0) return;
    const BoxcarArgs* cj = jobs + info[1];
    const int* prefix = prefix_base + info[2];
    for_each_claimed(prefix[njobs], queue, [&](int v) {
        const int jb = find_row_job(prefix, njobs, v);
        // The thread index, opaque to the compiler in every row: else it
        // keeps lane-dependent values of the row body live across rows.
        int tv = static_cast<int>(threadIdx.x);
        asm volatile("" : "+v"(tv));
        boxcar_row<NWT>(cj[jb], v - prefix[jb], sh, tv);
    });
}

__global__ void zero_u64_kernel(unsigned long long* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

__global__ void zero_counts_kernel(const BoxcarArgs* __restrict__ jobs, const int* __restrict__ njobs_p) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < *njobs_p && jobs[j].want_cands) *jobs[j].count = 0ull;
}

// ---------------------------------------------------------------------------

int boxcar_tmax_bytes(int nwt, int64_t nt) {
    const int64_t b = (nt + kBoxTile - 1) / kBoxTile * boxcar_nwt(nwt) * 4;
    return b <= kTileMaxLds ? static_cast<int>(b) : 0;
}

hipError_t launch_boxcar(const BoxcarArgs& a_in, hipStream_t stream) {
    BoxcarArgs a = a_in;
    if (a.want_cands) {
        hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, stream, a.count);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.ndm <= 0) return hipSuccess;
    const int grid = a.ndm;
    const int nwt = boxcar_nwt(a.ne);
    const int lds = boxcar_tmax_bytes(a.ne, a.nt);
    a.tmax_ok = lds > 0 ? 1 : 0;
    const int prof = prof_begin(TX_KERNEL_BOXCAR, stream);
    switch (nwt) {
        case 4: hipLaunchKernelGGL(boxcar_kernel<4>, dim3(grid), dim3(kThreads), lds, stream, a); break;
        case 8: hipLaunchKernelGGL(boxcar_kernel<8>, dim3(grid), dim3(kThreads), lds, stream, a); break;
        case 10: hipLaunchKernelGGL(boxcar_kernel<10>, dim3(grid), dim3(kThreads), lds, stream, a); break;
        case 12: hipLaunchKernelGGL(boxcar_kernel<12>, dim3(grid), dim3(kThreads), lds, stream, a); break;
        case 16: hipLaunchKernelGGL(boxcar_kernel<16>, dim3(grid), dim3(kThreads), lds, stream, a); break;
        default: hipLaunchKernelGGL(boxcar_kernel<32>, dim3(grid), dim3(kThreads), lds, stream, a); break;
    }
    const hipError_t e = hipGetLastError();
    prof_end(prof, stream);
    return e;
}

hipError_t launch_boxcar_batch(int nwt, int lds, const BatchRefs& r, int64_t rows, hipStream_t stream) {
    const BoxcarArgs* jobs = static_cast<const BoxcarArgs*>(r.jobs);
    void* args[] = {&jobs, const_cast<const int**>(&r.prefix), const_cast<const int**>(&r.info),
                    const_cast<uint32_t**>(&r.queue)};
    const void* fn;
    switch (boxcar_nwt(nwt)) {
        case 4: fn = reinterpret_cast<const void*>(&boxcar_batch_kernel<4>); break;
        case 8: fn = reinterpret_cast<const void*>(&boxcar_batch_kernel<8>); break;
        case 10: fn = reinterpret_cast<const void*>(&boxcar_batch_kernel<10>); break;
        case 12: fn = reinterpret_cast<const void*>(&boxcar_batch_kernel<12>); break;
        case 16: fn = reinterpret_cast<const void*>(&boxcar_batch_kernel<16>); break;
        default: fn = reinterpret_cast<const void*>(&boxcar_batch_kernel<32>); break;
    }
    int grid = resident_grid(fn, lds);
    if (grid <= 0) grid = 256 * 5;
    if (rows > 0 && rows < grid) grid = static_cast<int>(rows);
    const int prof = prof_begin(TX_KERNEL_BOXCAR, stream);
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, static_cast<size_t>(lds), stream);
    if (e == hipSuccess) e = hipGetLastError();
    prof_end(prof, stream);
    return e;
}

hipError_t launch_zero_counts(const BoxcarArgs* d_jobs, const int* d_njobs, int max_jobs, hipStream_t stream) {
    if (max_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_counts_kernel, dim3((max_jobs + 255) / 256), dim3(256), 0, stream, d_jobs, d_njobs);
    return hipGetLastError();
}

}  // namespace tx
