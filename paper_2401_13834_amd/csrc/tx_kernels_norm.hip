// Dedispersion of normalised data and the matched filter of float series
// (gfx950): the floating-point variant of the hot path, for blocks whose
// channels are normalised before dedispersion (Sec. 2.1).
//
// A channel's normalised sample is scale[c] * x - offset[c] (float32 scale
// and offset; unit-variance or inverse-variance weights).  The two stages are
// those of the integer path (same plan, same offsets), summed in float32:
//   B[j][s][u] = sum over ch in s of (scale x[ch][u + D(c_j, f_ch)] - offset),
//   Y[i][t]    = sum over s of B[j][s][t + D(dm_i, f_s) - D(c_j, f_s)].
// Stage 1 stages channel rows as bytes in LDS (shared by the workgroup's
// coarse trials) and each lane turns the bytes of its outputs into one fused
// multiply-add per channel; stage 2 stages float32 sub-band rows in LDS (any
// element shift is an aligned 4-byte read) and adds.  The matched filter
// reads each row twice: once for its float64 moments, once for float64
// running sums per tile, S/N of every (start, width) in float64, the per-width
// best and the thresholded list.  Every channel term is rounded to float32
// once (a fused multiply-add) and then added, so a float32 output differs
// from the exact sum by at most (m + nsub + 1) 2^-24 times the sum of the
// absolute terms.
#include <algorithm>

#include "tx_internal.h"

#pragma clang fp contract(off)

namespace tx {

namespace {

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int block_max_i(int v, int* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    v = max(max(red[0], red[1]), max(red[2], red[3]));
    __syncthreads();
    return v;
}

// Byte k of w as a float (one v_cvt_f32_ubyteN).
__device__ __forceinline__ float byte_f(uint32_t w, int k) { return static_cast<float>((w >> (8 * k)) & 0xFFu); }

}  // namespace

// ---------------------------------------------------------------------------
// Stage 1.  Workgroup = (sub-band s, kNormJ coarse trials, kNormTT1 outputs):
// the 4 wavefronts split the time tile, lane l of wave w owns the 8
// consecutive outputs 8 (64 w + l) ..; every lane accumulates all the
// workgroup's trials.  Channel rows are staged, a round of rows at a time, as
// bytes from the first trial's shift rounded down to 16 bytes.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void stage1_norm_kernel(Stage1NormArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr int J = kNormJ;
    constexpr int TT = kNormTT1;
    const int tile = static_cast<int>(blockIdx.x);
    const int jc = tile % a.n_jchunks;
    const int rest = tile / a.n_jchunks;
    const int tt = rest % a.n_ttiles;
    const int s = rest / a.n_ttiles;
    const int j0 = jc * J;
    const int jl = min(j0 + J, a.ngroups) - 1;
    const int u0 = tt * TT;
    const int tid = threadIdx.x;
    const int ch0 = s * a.m;
    const TX_GLOBAL int32_t* __restrict__ dT = to_global(a.dT);
    const size_t gp = static_cast<size_t>(a.gpad);
    int* red = reinterpret_cast<int*>(lds);

    int sp = 0;
    for (int c = tid; c < a.m; c += kThreads) {
        const TX_GLOBAL int32_t* r = dT + static_cast<size_t>(ch0 + c) * gp;
        sp = max(sp, r[jl] - (r[j0] & ~15));
    }
    sp = uniform_i(block_max_i(sp, red));
    const int rowbytes = (sp + TT + 4 + 15) & ~15;        // staged bytes per row (one dword past the last output)

    // Tables at the top of LDS: per (channel, trial) the shift from the
    // channel's staging start; per channel its start.
    const int tab_off = (a.lds_bytes - ((a.m * (J + 1) * 4 + 15) & ~15)) & ~15;
    int32_t* tab = reinterpret_cast<int32_t*>(lds + tab_off);   // [m][J]
    int32_t* st0 = tab + a.m * J;                                 // [m]
    for (int t = tid; t < a.m * J; t += kThreads) {
        const int c = t / J, k = t - c * J;
        const TX_GLOBAL int32_t* r = dT + static_cast<size_t>(ch0 + c) * gp;
        tab[t] = r[min(j0 + k, jl)] - (r[j0] & ~15);
    }
    for (int c = tid; c < a.m; c += kThreads) st0[c] = dT[static_cast<size_t>(ch0 + c) * gp + j0] & ~15;
    const int nch = max(1, min(a.m, tab_off / rowbytes));
    __syncthreads();

    float acc[J][8];
#pragma unroll
    for (int k = 0; k < J; ++k)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[k][q] = 0.0f;
    const int ob = 8 * tid;                                       // this lane's first output
    const TX_GLOBAL float* __restrict__ scale = to_global(a.scale);
    const TX_GLOBAL float* __restrict__ offset = to_global(a.offset);

    for (int cb = 0; cb < a.m; cb += nch) {
        const int nc = min(nch, a.m - cb);
        // Stage rows [cb, cb + nc): 16-byte pieces where the whole piece is
        // valid, byte by byte at the row's end; zeros past it.
        for (int idx = tid; idx < nc * (rowbytes >> 4); idx += kThreads) {
            const int c = idx / (rowbytes >> 4), piece = idx - c * (rowbytes >> 4);
            const int64_t start = static_cast<int64_t>(u0) + st0[cb + c] + 16 * piece;
            const TX_GLOBAL uint8_t* row = to_global(a.x) + static_cast<size_t>(ch0 + cb + c) * a.x_pitch;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (start + 16 <= a.x_len) {
                v = *reinterpret_cast<const TX_GLOBAL uint4*>(row + start);
            } else if (start < a.x_len) {
                uint32_t d[4] = {0u, 0u, 0u, 0u};
                for (int b = 0; b < static_cast<int>(a.x_len - start); ++b)
                    d[b >> 2] |= static_cast<uint32_t>(row[start + b]) << (8 * (b & 3));
                v = make_uint4(d[0], d[1], d[2], d[3]);
            }
            *reinterpret_cast<uint4*>(lds + c * rowbytes + 16 * piece) = v;
        }
        __syncthreads();
        for (int c = 0; c < nc; ++c) {
            const float sc = scale[ch0 + cb + c];
            const float of = -offset[ch0 + cb + c];
            const uint8_t* row = lds + c * rowbytes;
#pragma unroll
            for (int k = 0; k < J; ++k) {
                const int e = uniform_i(tab[(cb + c) * J + k]) + ob;   // byte of output ob for trial k
                const uint32_t* p = reinterpret_cast<const uint32_t*>(row + (e & ~3));
                const uint32_t sh = static_cast<uint32_t>(e & 3);
                const uint32_t w0 = p[0], w1 = p[1], w2 = p[2];
                const uint32_t a0 = __builtin_amdgcn_alignbyte(w1, w0, sh);
                const uint32_t a1 = __builtin_amdgcn_alignbyte(w2, w1, sh);
                // the channel's normalised sample, rounded once, then added
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    acc[k][q] += __builtin_fmaf(byte_f(a0, q), sc, of);
                    acc[k][q + 4] += __builtin_fmaf(byte_f(a1, q), sc, of);
                }
            }
        }
        __syncthreads();
    }
    for (int k = 0; k < J; ++k) {
        const int j = j0 + k;
        if (j > jl) break;
        TX_GLOBAL float* out = to_global(a.B) + (static_cast<size_t>(j) * a.nsub + s) * a.B_pitch + u0 + ob;
        *reinterpret_cast<TX_GLOBAL float4*>(out) = make_float4(acc[k][0], acc[k][1], acc[k][2], acc[k][3]);
        *reinterpret_cast<TX_GLOBAL float4*>(out + 4) = make_float4(acc[k][4], acc[k][5], acc[k][6], acc[k][7]);
    }
}

// ---------------------------------------------------------------------------
// Stage 2.  Workgroup = (group j, up to kNormIW of its trials, kNormTT2
// outputs); lane tid owns the outputs t0 + tid + 256 k (k < 4), so every LDS
// read of a trial is 64 consecutive floats of one row (no bank conflicts at
// any shift).  Sub-band rows are staged a round at a time.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void stage2_norm_kernel(Stage2NormArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr int IW = kNormIW;
    constexpr int TT = kNormTT2;
    const int tile = static_cast<int>(blockIdx.x);
    const int ic = tile % a.n_ichunks;
    const int rest = tile / a.n_ichunks;
    const int tt = rest % a.n_ttiles;
    const int j = rest / a.n_ttiles;
    const int i0 = j * a.g + ic * IW;
    const int iend = min((j + 1) * a.g, a.ndm);
    const int ni = min(IW, iend - i0);
    if (ni <= 0) return;
    const int il = i0 + ni - 1;
    const int t0 = tt * TT;
    const int tid = threadIdx.x;
    const TX_GLOBAL int32_t* __restrict__ rT = to_global(a.rT);
    const size_t dp = static_cast<size_t>(a.dpad);
    int* red = reinterpret_cast<int*>(lds);

    int sp = 0;
    for (int s = tid; s < a.nsub; s += kThreads) {
        const TX_GLOBAL int32_t* r = rT + static_cast<size_t>(s) * dp;
        sp = max(sp, r[il] - (r[i0] & ~3));
    }
    sp = uniform_i(block_max_i(sp, red));
    const int rowf = (sp + TT + 3) & ~3;                  // staged floats per row
    const int tab_off = (a.lds_bytes - ((IW * a.nsub * 4 + 15) & ~15)) & ~15;
    int32_t* tab = reinterpret_cast<int32_t*>(lds + tab_off);   // [nsub][IW]: shift from the staged start
    for (int t = tid; t < IW * a.nsub; t += kThreads) {
        const int s = t / IW, k = t - s * IW;
        const TX_GLOBAL int32_t* r = rT + static_cast<size_t>(s) * dp;
        tab[t] = r[i0 + min(k, ni - 1)] - (r[i0] & ~3);
    }
    const int nsb = max(1, min(a.nsub, tab_off / (rowf * 4)));
    __syncthreads();

    float acc[IW][4];
#pragma unroll
    for (int k = 0; k < IW; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[k][q] = 0.0f;
    const TX_GLOBAL float* Bj = to_global(a.B) + static_cast<size_t>(j) * a.nsub * a.B_pitch;
    float* rows = reinterpret_cast<float*>(lds);
    for (int sb = 0; sb < a.nsub; sb += nsb) {
        const int ns = min(nsb, a.nsub - sb);
        for (int idx = tid; idx < ns * (rowf >> 2); idx += kThreads) {
            const int r = idx / (rowf >> 2), piece = idx - r * (rowf >> 2);
            const int s = sb + r;
            const TX_GLOBAL float* src = Bj + static_cast<size_t>(s) * a.B_pitch + t0 + (rT[static_cast<size_t>(s) * dp + i0] & ~3);
            *reinterpret_cast<float4*>(rows + r * rowf + 4 * piece) =
                *reinterpret_cast<const TX_GLOBAL float4*>(src + 4 * piece);
        }
        __syncthreads();
        for (int r = 0; r < ns; ++r) {
            const float* row = rows + r * rowf + tid;
#pragma unroll
            for (int k = 0; k < IW; ++k) {
                const int e = uniform_i(tab[(sb + r) * IW + k]);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[k][q] += row[e + 256 * q];
            }
        }
        __syncthreads();
    }
    for (int k = 0; k < ni; ++k) {
        TX_GLOBAL float* out = to_global(a.Y) + static_cast<size_t>(i0 + k) * a.y_pitch;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t t = t0 + tid + 256 * q;
            if (t < a.nt) out[t] = acc[k][q];
        }
    }
}

// ---------------------------------------------------------------------------
// Matched filter of float series.  One workgroup per row: float64 sum and
// sum of squares give the mean and sigma; then per tile of kBoxTile starts,
// float64 running sums in LDS, and every start's S/N at every width (thread
// tid owns the starts tid + 256 m).  Per width the largest S/N (earliest
// start); across widths the largest (ties to the smaller width); a start
// whose best S/N reaches gamma is listed.  NWT: widths the instance holds
// (slots past the row's widths repeat its last width).
// ---------------------------------------------------------------------------
struct NormBoxShared {
    double P[kBoxTile + TX_MAX_WIDTH + 16];
    double wsum[kWaves];
    double red1[kWaves], red2[kWaves];
    double bs[kWaves][TX_MAX_WIDTHS];
    int32_t bt[kWaves][TX_MAX_WIDTHS];
    int32_t wd[TX_MAX_WIDTHS];
    double rs[TX_MAX_WIDTHS];
    double mean, inv;
    int state;
};

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int NWT>
__global__ __launch_bounds__(kThreads) void boxcar_norm_kernel(BoxcarNormArgs a) {
    __shared__ NormBoxShared sh;
    const int row = static_cast<int>(blockIdx.x);
    if (row >= a.ndm) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int T = a.nt;
    const TX_GLOBAL float* __restrict__ y = to_global(a.y) + static_cast<size_t>(row) * a.pitch;
    if (tid < NWT) {
        int32_t w = 0;
        double r = 0.0;
#pragma unroll
        for (int k = 0; k < NWT; ++k)
            if (k == tid) {
                w = a.widths[k];
                r = a.rsw[k];
            }
        sh.wd[tid] = w;
        sh.rs[tid] = r;
    }

    // moments
    double s1 = 0.0, s2 = 0.0;
    for (int t = tid; t < T; t += kThreads) {
        const double v = static_cast<double>(y[t]);
        s1 += v;
        s2 += v * v;
    }
    s1 = wave_sum_d(s1);
    s2 = wave_sum_d(s2);
    if (lane == 0) {
        sh.red1[wave] = s1;
        sh.red2[wave] = s2;
    }
    __syncthreads();
    if (tid == 0) {
        const double S1 = (sh.red1[0] + sh.red1[1]) + (sh.red1[2] + sh.red1[3]);
        const double S2 = (sh.red2[0] + sh.red2[1]) + (sh.red2[2] + sh.red2[3]);
        const double mean = S1 / static_cast<double>(T);
        const double var = S2 / static_cast<double>(T) - mean * mean;
        if (a.fixed) {                                  // given noise statistics
            sh.mean = a.fixed_mean;
            sh.inv = 1.0 / a.fixed_sigma;
            sh.state = 0;
        } else {
            sh.mean = mean;
            sh.inv = var > 0.0 ? 1.0 / __builtin_sqrt(var) : 0.0;
            sh.state = var > 0.0 ? 0 : 1;
        }
    }
    __syncthreads();
    if (sh.state != 0) {
        if (tid == 0 && a.want_peaks) {
            to_global(a.snr)[row] = 0.0;
            to_global(a.width)[row] = a.w_first;
            to_global(a.time)[row] = 0;
        }
        return;
    }
    const double mean = sh.mean, inv = sh.inv;
    double bs[NWT];
    int32_t bt[NWT];
#pragma unroll
    for (int i = 0; i < NWT; ++i) {
        bs[i] = -__builtin_inf();
        bt[i] = 0;
    }
    const int ntiles = (T + kBoxTile - 1) / kBoxTile;
    const int L = kBoxTile + a.wmax;
    for (int tile = 0; tile < ntiles; ++tile) {
        const int t0 = tile * kBoxTile;
        // Running sums P[e] = sum of y[t0 .. t0 + e), e <= L (zeros past T):
        // each thread sums 24 consecutive samples; a wavefront scan and the
        // earlier wavefronts' totals give its base.
        constexpr int kPer = 24;
        const int e0 = kPer * tid;
        double v[kPer];
        double run = 0.0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int e = e0 + k;
            const int64_t t = static_cast<int64_t>(t0) + e;
            v[k] = (e < L && t < T) ? static_cast<double>(y[t]) : 0.0;
            run += v[k];
        }
        double incl = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double up = __shfl_up(incl, o);
            if (lane >= o) incl += up;
        }
        if (lane == 63) sh.wsum[wave] = incl;
        __syncthreads();
        double base = incl - run;
        for (int w2 = 0; w2 < wave; ++w2) base += sh.wsum[w2];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (e0 + k <= L) sh.P[e0 + k] = base;
            base += v[k];
        }
        __syncthreads();
#pragma unroll 1
        for (int m = 0; m < kBoxTile / kThreads; ++m) {
            const int e = tid + 256 * m;
            const int t = t0 + e;
            if (t >= T) break;
            const double pe = sh.P[e];
            double best = -__builtin_inf();
            int bw = -1;
#pragma unroll
            for (int i = 0; i < NWT; ++i) {
                const int w = sh.wd[i];
                if (i >= a.ne || t + w > T) continue;
                const double S = sh.P[e + w] - pe;
                const double sn = ((S - static_cast<double>(w) * mean) * inv) * sh.rs[i];
                if (sn > bs[i]) {                          // starts increase: the first maximum stays
                    bs[i] = sn;
                    bt[i] = t;
                }
                if (bw < 0 || sn > best) {
                    best = sn;
                    bw = w;
                }
            }
            if (a.want_cands && bw > 0 && best >= a.gamma) {
                const unsigned long long slot = atomicAdd(a.count, 1ull);
                if (static_cast<long long>(slot) < a.cap) {
                    tx_cand c;
                    c.dm_index = row;
                    c.width = bw;
                    c.time = t;
                    c.snr = best;
                    to_global(a.cands)[slot] = c;
                }
            }
        }
        __syncthreads();
    }
    // Per width: the largest S/N over the workgroup, the earliest start on ties.
#pragma unroll
    for (int i = 0; i < NWT; ++i) {
        double s = bs[i];
        int32_t t = bt[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double s2o = __shfl_xor(s, o);
            const int32_t t2o = __shfl_xor(t, o);
            if (s2o > s || (s2o == s && t2o < t)) {
                s = s2o;
                t = t2o;
            }
        }
        if (lane == 0) {
            sh.bs[wave][i] = s;
            sh.bt[wave][i] = t;
        }
    }
    __syncthreads();
    if (tid == 0 && a.want_peaks) {
        double best = 0.0;
        int bw = -1;
        int64_t btm = 0;
        for (int i = 0; i < a.ne; ++i) {
            double s = sh.bs[0][i];
            int32_t t = sh.bt[0][i];
            for (int w2 = 1; w2 < kWaves; ++w2)
                if (sh.bs[w2][i] > s || (sh.bs[w2][i] == s && sh.bt[w2][i] < t)) {
                    s = sh.bs[w2][i];
                    t = sh.bt[w2][i];
                }
            if (s == -__builtin_inf()) continue;
            if (bw < 0 || s > best) {
                best = s;
                bw = sh.wd[i];
                btm = t;
            }
        }
        if (bw < 0) {
            best = 0.0;
            bw = a.w_first;
            btm = 0;
        }
        to_global(a.snr)[row] = best;
        to_global(a.width)[row] = bw;
        to_global(a.time)[row] = btm;
    }
}

__global__ void zero_count_norm_kernel(unsigned long long* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

// ---------------------------------------------------------------------------

NormGeom norm_geometry(const tx_plan_s* p, int64_t nt) {
    NormGeom g{};
    g.n_ttiles2 = static_cast<int32_t>((nt + kNormTT2 - 1) / kNormTT2);
    g.n_ichunks = (p->g + kNormIW - 1) / kNormIW;
    g.n_jchunks = (p->ngroups + kNormJ - 1) / kNormJ;
    // stage 2 stages floats [start, start + rowf) of a series, start <= last
    // tile start + max extent; rowf <= spread + TT + 3
    const int sp2 = plan_spread2(p, kNormIW) + 3;
    const int64_t need = static_cast<int64_t>(std::max(g.n_ttiles2 - 1, 0)) * kNormTT2 + p->max_extent + sp2 + kNormTT2 + 4;
    g.B_pitch = (std::max<int64_t>(need, nt + p->max_extent) + kNormTT1 - 1) / kNormTT1 * kNormTT1;
    g.n_ttiles1 = static_cast<int32_t>(g.B_pitch / kNormTT1);
    g.ws_bytes = (static_cast<int64_t>(p->ngroups) * p->nsub * g.B_pitch * 4 + 255) / 256 * 256;
    const int sp1 = plan_spread1(p, kNormJ) + 15;
    const int row1 = (sp1 + kNormTT1 + 4 + 15) & ~15;
    g.lds1 = std::max(kNormLds, row1 + ((p->m * (kNormJ + 1) * 4 + 15) & ~15) + 64);
    const int row2 = ((sp2 + kNormTT2 + 3) & ~3) * 4;
    g.lds2 = std::max(kNormLds, row2 + ((kNormIW * p->nsub * 4 + 15) & ~15) + 64);
    g.ok = g.lds1 <= device_max_lds() && g.lds2 <= device_max_lds();
    return g;
}

static hipError_t launch_lds(const void* fn, int grid, int lds, void** args, hipStream_t st) {
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        (void)hipGetLastError();
    }
    const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, static_cast<size_t>(lds), st);
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_dedisperse_norm(const tx_plan_s* p, const NormGeom& g, const uint8_t* d_in, int64_t in_pitch,
                                  int64_t nt, const float* scale, const float* offset, float* d_out,
                                  int64_t out_pitch, float* d_B, hipStream_t stream) {
    if (!g.ok) return hipErrorInvalidValue;
    Stage1NormArgs a1{};
    a1.x = d_in;
    a1.x_pitch = in_pitch;
    a1.x_len = nt + p->overlap;
    a1.scale = scale;
    a1.offset = offset;
    a1.B = d_B;
    a1.B_pitch = g.B_pitch;
    a1.dT = p->d_dT;
    a1.gpad = p->gpad;
    a1.nsub = p->nsub;
    a1.m = p->m;
    a1.ngroups = p->ngroups;
    a1.n_jchunks = g.n_jchunks;
    a1.n_ttiles = g.n_ttiles1;
    a1.lds_bytes = g.lds1;
    Stage2NormArgs a2{};
    a2.B = d_B;
    a2.B_pitch = g.B_pitch;
    a2.Y = d_out;
    a2.y_pitch = out_pitch;
    a2.nt = nt;
    a2.rT = p->d_rT;
    a2.dpad = p->dpad;
    a2.ndm = p->ndm;
    a2.nsub = p->nsub;
    a2.g = p->g;
    a2.ngroups = p->ngroups;
    a2.n_ichunks = g.n_ichunks;
    a2.n_ttiles = g.n_ttiles2;
    a2.lds_bytes = g.lds2;
    void* v1[] = {&a1};
    const int64_t grid1 = static_cast<int64_t>(p->nsub) * g.n_ttiles1 * g.n_jchunks;
    const int64_t grid2 = static_cast<int64_t>(p->ngroups) * g.n_ichunks * g.n_ttiles2;
    if (grid1 > INT32_MAX || grid2 > INT32_MAX) return hipErrorInvalidValue;
    int prof = prof_begin(TX_KERNEL_STAGE1, stream);
    hipError_t e = launch_lds(reinterpret_cast<const void*>(&stage1_norm_kernel), static_cast<int>(grid1), g.lds1, v1,
                              stream);
    prof_end(prof, stream);
    if (e != hipSuccess) return e;
    void* v2[] = {&a2};
    prof = prof_begin(TX_KERNEL_STAGE2, stream);
    e = launch_lds(reinterpret_cast<const void*>(&stage2_norm_kernel), static_cast<int>(grid2), g.lds2, v2, stream);
    prof_end(prof, stream);
    return e;
}

hipError_t launch_boxcar_norm(const BoxcarNormArgs& a, hipStream_t stream) {
    if (a.want_cands) {
        hipLaunchKernelGGL(zero_count_norm_kernel, dim3(1), dim3(64), 0, stream, a.count);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (a.ndm <= 0) return hipSuccess;
    const int prof = prof_begin(TX_KERNEL_BOXCAR, stream);
    switch (boxcar_nwt(a.ne)) {
        case 4: hipLaunchKernelGGL(boxcar_norm_kernel<4>, dim3(a.ndm), dim3(kThreads), 0, stream, a); break;
        case 8: hipLaunchKernelGGL(boxcar_norm_kernel<8>, dim3(a.ndm), dim3(kThreads), 0, stream, a); break;
        case 10: hipLaunchKernelGGL(boxcar_norm_kernel<10>, dim3(a.ndm), dim3(kThreads), 0, stream, a); break;
        case 12: hipLaunchKernelGGL(boxcar_norm_kernel<12>, dim3(a.ndm), dim3(kThreads), 0, stream, a); break;
        case 16: hipLaunchKernelGGL(boxcar_norm_kernel<16>, dim3(a.ndm), dim3(kThreads), 0, stream, a); break;
        default: hipLaunchKernelGGL(boxcar_norm_kernel<32>, dim3(a.ndm), dim3(kThreads), 0, stream, a); break;
    }
    const hipError_t e = hipGetLastError();
    prof_end(prof, stream);
    return e;
}

}  // namespace tx
