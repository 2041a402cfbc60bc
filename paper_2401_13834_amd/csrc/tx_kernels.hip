// HIP kernels for gfx950 (MI355X): two-stage sub-band dedispersion and the
// boxcar matched filter.
//
// Layout: filterbank rows are channel-major uint8; first-stage series are
// uint16 [group][sub-band][time]; the output is int32 [trial][time].
// All sums are integer and exact, so any tiling gives bit-identical results.
//
// Both dedispersion stages are shift-and-add with a per-(trial, row) shift
// that is the same for every lane of a wavefront: lanes walk the time axis,
// so a wave reads a contiguous LDS window at one shift and the shift, its
// byte misalignment and the byte-select patterns live in scalar registers.
#include <algorithm>

#include "tx_internal.h"

#pragma clang fp contract(off)

namespace tx {

__device__ __forceinline__ uint32_t perm_b32(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}
__device__ __forceinline__ uint32_t align_b32(uint32_t hi, uint32_t lo, uint32_t nbytes) {
    return __builtin_amdgcn_alignbyte(hi, lo, nbytes);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Consecutive workgroup ids are dealt round-robin to the 8 XCDs; give each XCD
// a contiguous range of tiles so that tiles sharing input rows share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int total) {
    const int nx = 8;
    int x = bid % nx, k = bid / nx;
    int q = total / nx, r = total % nx;
    return x * q + min(x, r) + k;
}

// ---------------------------------------------------------------------------
// Stage 1: B[j][s][u] = sum over ch in s of x[ch][u + D(c_j, f_ch)].
//
// Workgroup = (sub-band s, J1 coarse trials, TT1 outputs).  Channel rows are
// staged in LDS, each starting at its own shift for the first trial of the
// workgroup (16-byte aligned down; the remainder joins the per-trial shift).
// Lane l of a wave owns output dwords l + 64 q (4 outputs each).  For a shift
// of k bytes past a dword boundary, alignbyte picks the 4 input bytes and a
// byte permute picks bytes 1 and 3 into 16-bit lanes.  Two accumulators per
// dword: "full" adds the 4 bytes as one 32-bit word (carries cross bytes) and
// "odd" holds bytes 1 and 3 as 16-bit sums; at the end
// full - (odd << 8) = (sum b0) | (sum b2) << 16 exactly, because every 16-bit
// sum of <= 256 bytes is < 2^16.
// ---------------------------------------------------------------------------
template <int Q, int JW>
__global__ __launch_bounds__(kThreads) void stage1_kernel(Stage1Args a) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int total = a.nsub * a.n_ttiles * a.n_jchunks;
    const int tile = xcd_tile(blockIdx.x, total);
    const int jc = tile % a.n_jchunks;
    const int rest = tile / a.n_jchunks;
    const int tt = rest % a.n_ttiles;
    const int s = rest / a.n_ttiles;
    const int j0 = jc * (JW * kWaves);
    const int64_t u0 = static_cast<int64_t>(tt) * (256 * Q);
    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);
    const int jw0 = j0 + wave * JW;
    const int ch0 = s * a.m;
    const int32_t* __restrict__ d0 = a.dcc + static_cast<size_t>(j0) * a.nchan;

    uint32_t full[JW][Q], odd[JW][Q];
#pragma unroll
    for (int jj = 0; jj < JW; ++jj)
#pragma unroll
        for (int q = 0; q < Q; ++q) full[jj][q] = odd[jj][q] = 0u;

    const int vpr = a.lds_row >> 4;
    for (int cb = 0; cb < a.m; cb += a.cchunk) {
        const int nc = min(a.cchunk, a.m - cb);
        for (int v = threadIdx.x; v < nc * vpr; v += kThreads) {
            const int c = v / vpr;
            const int off = (v - c * vpr) << 4;
            const int ch = ch0 + cb + c;
            const int64_t start = u0 + d0[ch];
            const int64_t pos = (start & ~int64_t(15)) + off;
            const uint8_t* row = a.x + static_cast<size_t>(ch) * a.x_pitch;
            uint4 val;
            if (pos + 16 <= a.x_len) {
                val = *reinterpret_cast<const uint4*>(row + pos);
            } else {
                uint32_t w[4] = {0u, 0u, 0u, 0u};
                for (int b = 0; b < 16; ++b)
                    if (pos + b < a.x_len) w[b >> 2] |= static_cast<uint32_t>(row[pos + b]) << (8 * (b & 3));
                val = make_uint4(w[0], w[1], w[2], w[3]);
            }
            *reinterpret_cast<uint4*>(lds + c * a.lds_row + off) = val;
        }
        __syncthreads();
        for (int c = 0; c < nc; ++c) {
            const int ch = ch0 + cb + c;
            const int base = uniform(d0[ch]);
            const int mis = static_cast<int>((u0 + base) & 15);
            const uint8_t* rowp = lds + c * a.lds_row;
#pragma unroll
            for (int jj = 0; jj < JW; ++jj) {
                const int j = jw0 + jj;
                if (j < a.ngroups) {
                    const int sh = uniform(a.dcc[static_cast<size_t>(j) * a.nchan + ch]) - base + mis;
                    const uint32_t k = static_cast<uint32_t>(sh & 3);
                    const uint32_t sel = 0x0C030C01u + k * 0x00010001u;
                    const uint32_t* w = reinterpret_cast<const uint32_t*>(rowp + (sh & ~3)) + lane;
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const uint32_t lo = w[64 * q];
                        const uint32_t hi = w[64 * q + 1];
                        full[jj][q] += align_b32(hi, lo, k);
                        odd[jj][q] += perm_b32(hi, lo, sel);
                    }
                }
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int jj = 0; jj < JW; ++jj) {
        const int j = jw0 + jj;
        if (j < a.ngroups) {
            uint16_t* out = a.B + (static_cast<size_t>(j) * a.nsub + s) * a.B_pitch + u0;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const uint32_t even = full[jj][q] - (odd[jj][q] << 8);
                const uint32_t w01 = perm_b32(odd[jj][q], even, 0x05040100u);
                const uint32_t w23 = perm_b32(odd[jj][q], even, 0x07060302u);
                *reinterpret_cast<uint2*>(out + 4 * (lane + 64 * q)) = make_uint2(w01, w23);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Stage 2: Y[i][t] = sum over s of B[j][s][t + rel(i, s)],
// rel(i, s) = D(dm_i, f_s) - D(c_j, f_s).
//
// Workgroup = (group j, IW fine trials of it, TT2 outputs); the 4 waves split
// the time tile and each handles all IW trials.  Sub-band rows are staged in
// LDS starting at the shift of the chunk's first trial.  Lane l owns output
// pairs (dwords of two uint16) l + 64 q of its wave's share.  Pairs are summed
// as packed 16-bit lanes of one 32-bit word for `flush` sub-bands (exact, as
// flush * 255 * m < 2^16) and then widened into two int32 accumulators.
// ---------------------------------------------------------------------------
template <int IW, int Q>
__global__ __launch_bounds__(kThreads) void stage2_kernel(Stage2Args a) {
    extern __shared__ __align__(16) uint8_t lds_raw[];
    uint16_t* lds = reinterpret_cast<uint16_t*>(lds_raw);
    const int total = a.ngroups * a.n_ichunks * a.n_ttiles;
    const int tile = xcd_tile(blockIdx.x, total);
    const int ic = tile % a.n_ichunks;
    const int rest = tile / a.n_ichunks;
    const int tt = rest % a.n_ttiles;
    const int j = rest / a.n_ttiles;
    const int i0 = j * a.g + ic * IW;
    const int iend = min((j + 1) * a.g, a.ndm);
    const int ni = min(IW, iend - i0);
    if (ni <= 0) return;
    constexpr int TTW = 128 * Q;                  // outputs per wave
    const int64_t t0 = static_cast<int64_t>(tt) * (TTW * kWaves);
    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);
    const int32_t* __restrict__ r0 = a.rel + static_cast<size_t>(i0) * a.nsub;

    uint32_t acc[IW][Q], lo[IW][Q], hi[IW][Q];
#pragma unroll
    for (int ii = 0; ii < IW; ++ii)
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[ii][q] = lo[ii][q] = hi[ii][q] = 0u;
    int pending = 0;

    const int vpr = a.lds_row >> 3;               // 16-byte vectors per staged row
    const uint16_t* Bj = a.B + static_cast<size_t>(j) * a.nsub * a.B_pitch;
    for (int sb = 0; sb < a.nsub; sb += a.schunk) {
        const int ns = min(a.schunk, a.nsub - sb);
        for (int v = threadIdx.x; v < ns * vpr; v += kThreads) {
            const int r = v / vpr;
            const int off = (v - r * vpr) << 3;
            const int s = sb + r;
            const int64_t start = t0 + r0[s];
            const int64_t pos = (start & ~int64_t(7)) + off;
            const uint4 val = *reinterpret_cast<const uint4*>(Bj + static_cast<size_t>(s) * a.B_pitch + pos);
            *reinterpret_cast<uint4*>(lds + r * a.lds_row + off) = val;
        }
        __syncthreads();
        for (int r = 0; r < ns; ++r) {
            const int s = sb + r;
            const int base = uniform(r0[s]);
            const int mis = static_cast<int>((t0 + base) & 7);
            const uint32_t* roww = reinterpret_cast<const uint32_t*>(lds + r * a.lds_row) + wave * (64 * Q) + lane;
#pragma unroll
            for (int ii = 0; ii < IW; ++ii) {
                if (ii < ni) {
                    const int e = uniform(a.rel[static_cast<size_t>(i0 + ii) * a.nsub + s]) - base + mis;
                    const uint32_t k = static_cast<uint32_t>((e & 1) << 1);
                    const uint32_t* w = roww + (e >> 1);
#pragma unroll
                    for (int q = 0; q < Q; ++q) acc[ii][q] += align_b32(w[64 * q + 1], w[64 * q], k);
                }
            }
            if (++pending == a.flush) {
#pragma unroll
                for (int ii = 0; ii < IW; ++ii)
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        lo[ii][q] += acc[ii][q] & 0xFFFFu;
                        hi[ii][q] += acc[ii][q] >> 16;
                        acc[ii][q] = 0u;
                    }
                pending = 0;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int ii = 0; ii < IW; ++ii)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            lo[ii][q] += acc[ii][q] & 0xFFFFu;
            hi[ii][q] += acc[ii][q] >> 16;
        }

#pragma unroll
    for (int ii = 0; ii < IW; ++ii) {
        if (ii < ni) {
            int32_t* out = a.Y + static_cast<size_t>(i0 + ii) * a.y_pitch;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int64_t t = t0 + 2 * (wave * (64 * Q) + lane + 64 * q);
                if (t + 1 < a.nt) {
                    *reinterpret_cast<int2*>(out + t) = make_int2(static_cast<int32_t>(lo[ii][q]),
                                                                  static_cast<int32_t>(hi[ii][q]));
                } else if (t < a.nt) {
                    out[t] = static_cast<int32_t>(lo[ii][q]);
                }
            }
        }
    }
}

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

// ---------------------------------------------------------------------------
// Host-side launch helpers.
// ---------------------------------------------------------------------------
static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

static int pick_iw(int32_t g) {
    static const int cands[] = {16, 13, 8, 4, 2, 1};
    int best = 1;
    int64_t best_cost = INT64_MAX;
    for (int iw : cands) {
        int64_t cost = (g + iw - 1) / iw * static_cast<int64_t>(iw);
        if (cost < best_cost) {
            best_cost = cost;
            best = iw;
        }
    }
    return best;
}

static int32_t stage2_spread(const tx_plan_s* p, int iw) {
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
    return sp;
}

DedispGeom dedisp_geometry(const tx_plan_s* p, int64_t nt) {
    DedispGeom g{};
    const int iw = pick_iw(p->g);
    const int32_t sp2 = stage2_spread(p, iw);
    g.n_ttiles2 = static_cast<int32_t>((nt + TT2 - 1) / TT2);
    g.lds2_row = static_cast<int32_t>(round_up(TT2 + sp2 + 16, 8));
    g.schunk = std::max(1, std::min(p->nsub, kLdsBudget / (2 * g.lds2_row)));
    const int64_t need = std::max<int64_t>(static_cast<int64_t>(std::max(g.n_ttiles2 - 1, 0)) * TT2 +
                                               p->max_extent + g.lds2_row,
                                           nt + p->max_extent);
    g.B_pitch = round_up(std::max<int64_t>(need, 1), TT1);
    g.n_ttiles1 = static_cast<int32_t>(g.B_pitch / TT1);
    g.lds1_row = static_cast<int32_t>(round_up(TT1 + p->spread1 + 24, 16));
    g.cchunk = std::max(1, std::min(p->m, kLdsBudget / g.lds1_row));
    g.ws_bytes = round_up(static_cast<int64_t>(p->ngroups) * p->nsub * g.B_pitch * 2, 256);
    return g;
}

template <int IW>
static hipError_t launch_stage2_iw(const Stage2Args& a, int grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((stage2_kernel<IW, Q2>), dim3(grid), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_dedisperse(const tx_plan_s* p, const DedispGeom& geo, const uint8_t* d_in,
                             int64_t in_pitch, int64_t nt, int32_t* d_out, int64_t out_pitch,
                             uint16_t* d_B, hipStream_t stream) {
    Stage1Args s1{};
    s1.x = d_in;
    s1.x_pitch = in_pitch;
    s1.x_len = nt + p->overlap;
    s1.B = d_B;
    s1.B_pitch = geo.B_pitch;
    s1.dcc = p->d_coarse_chan;
    s1.nchan = p->nchan;
    s1.nsub = p->nsub;
    s1.m = p->m;
    s1.ngroups = p->ngroups;
    s1.n_jchunks = (p->ngroups + J1 - 1) / J1;
    s1.n_ttiles = geo.n_ttiles1;
    s1.lds_row = geo.lds1_row;
    s1.cchunk = geo.cchunk;
    const int64_t grid1 = static_cast<int64_t>(s1.nsub) * s1.n_ttiles * s1.n_jchunks;
    const size_t lds1 = static_cast<size_t>(geo.cchunk) * geo.lds1_row;
    int prof = prof_begin(TX_KERNEL_STAGE1, stream);
    hipLaunchKernelGGL((stage1_kernel<Q1, J1W>), dim3(static_cast<uint32_t>(grid1)), dim3(kThreads), lds1, stream, s1);
    hipError_t e = hipGetLastError();
    prof_end(prof, stream);
    if (e != hipSuccess) return e;

    Stage2Args s2{};
    s2.B = d_B;
    s2.B_pitch = geo.B_pitch;
    s2.Y = d_out;
    s2.y_pitch = out_pitch;
    s2.nt = nt;
    s2.rel = p->d_rel;
    s2.ndm = p->ndm;
    s2.nsub = p->nsub;
    s2.g = p->g;
    s2.ngroups = p->ngroups;
    const int iw = pick_iw(p->g);
    s2.n_ichunks = (p->g + iw - 1) / iw;
    s2.n_ttiles = geo.n_ttiles2;
    s2.lds_row = geo.lds2_row;
    s2.schunk = geo.schunk;
    s2.flush = std::max(1, 65535 / (255 * p->m));
    const int64_t grid2 = static_cast<int64_t>(s2.ngroups) * s2.n_ichunks * s2.n_ttiles;
    const size_t lds2 = static_cast<size_t>(geo.schunk) * geo.lds2_row * 2;
    const int g2 = static_cast<int>(grid2);
    prof = prof_begin(TX_KERNEL_STAGE2, stream);
    switch (iw) {
        case 16: e = launch_stage2_iw<16>(s2, g2, lds2, stream); break;
        case 13: e = launch_stage2_iw<13>(s2, g2, lds2, stream); break;
        case 8: e = launch_stage2_iw<8>(s2, g2, lds2, stream); break;
        case 4: e = launch_stage2_iw<4>(s2, g2, lds2, stream); break;
        case 2: e = launch_stage2_iw<2>(s2, g2, lds2, stream); break;
        default: e = launch_stage2_iw<1>(s2, g2, lds2, stream); break;
    }
    prof_end(prof, stream);
    return e;
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
