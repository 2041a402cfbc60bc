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
// reads each row once (float64 moments and per-tile running sums, the largest
// window sum per width) and again only the tiles holding candidates.  Every
// channel term is rounded to float32 once (a fused multiply-add) and then
// added, so a float32 output differs from the exact sum by at most
// (m + nsub + 1) 2^-24 times the sum of the absolute terms.
#include <algorithm>

#include "tx_internal.h"

#pragma clang fp contract(off)

namespace tx {

namespace {

// Byte k of w as a float (one v_cvt_f32_ubyteN).
__device__ __forceinline__ float byte_f(uint32_t w, int k) { return static_cast<float>((w >> (8 * k)) & 0xFFu); }

}  // namespace

// ---------------------------------------------------------------------------
// Stage 1.  Workgroup = (sub-band s, J = 4 kNormJW coarse trials, TT =
// 256 kNormQ outputs): wave w owns trials j0 + w kNormJW .. and lane l the
// 4 kNormQ consecutive outputs from 4 kNormQ l.  A lane reads the kNormQ + 1
// input dwords of a (channel, trial) as paired 4-byte reads from one base
// (kNormQ odd: the lanes' addresses fall in distinct banks) and takes each
// output dword's 4 bytes with one byte align.  Channel rows are staged as
// bytes, from the first trial's shift rounded down to 16 bytes, by buffer
// loads straight into LDS (range-checked: zeros past a row's valid bytes),
// double-buffered where two rounds of rows fit.  A per-(channel, trial)
// table at the top of LDS holds each shift from the staging start.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void stage1_norm_kernel(Stage1NormArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr int Q = kNormQ;
    constexpr int JW = kNormJW;
    constexpr int J = JW * kWaves;
    constexpr int TT = 256 * Q;
    const int tile = xcd_tile(static_cast<int>(blockIdx.x), a.nsub * a.n_ttiles * a.n_jchunks);
    const int jc = tile % a.n_jchunks;
    const int rest = tile / a.n_jchunks;
    const int tt = rest % a.n_ttiles;
    const int s = rest / a.n_ttiles;
    const int j0 = jc * J;
    const int jl = min(j0 + J, a.ngroups) - 1;
    const int u0 = tt * TT;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const int ch0 = s * a.m;
    const TX_GLOBAL int32_t* __restrict__ dT = to_global(a.dT);
    const size_t gp = static_cast<size_t>(a.gpad);
    int* red = reinterpret_cast<int*>(lds);

    int sp = 0;
    for (int c = tid; c < a.m; c += kThreads) {
        const TX_GLOBAL int32_t* r = dT + static_cast<size_t>(ch0 + c) * gp;
        sp = max(sp, r[jl] - (r[j0] & ~15));
    }
    sp = uniform(block_max(sp, red));
    const int W = ((sp >> 2) + 64 * Q + 1 + 3) & ~3;      // dwords per staged row
    const int rowbytes = 4 * W;

    // Tables at the top of LDS: per (channel, trial) the shift from the
    // channel's staging start; per channel its start, scale and -offset.
    const int fix_off = (a.lds_bytes - ((a.m * (J + 3) * 4 + 15) & ~15)) & ~15;
    int32_t* tab = reinterpret_cast<int32_t*>(lds + fix_off);   // [m][J]
    int32_t* st0 = tab + a.m * J;                                 // [m]
    float* wsc = reinterpret_cast<float*>(st0 + a.m);             // [m]
    float* wof = wsc + a.m;                                       // [m]
    for (int t = tid; t < a.m * J; t += kThreads) {
        const int c = t / J, k = t - c * J;
        const TX_GLOBAL int32_t* r = dT + static_cast<size_t>(ch0 + c) * gp;
        tab[t] = r[min(j0 + k, jl)] - (r[j0] & ~15);
    }
    for (int c = tid; c < a.m; c += kThreads) {
        st0[c] = dT[static_cast<size_t>(ch0 + c) * gp + j0] & ~15;
        wsc[c] = to_global(a.scale)[ch0 + c];
        wof[c] = -to_global(a.offset)[ch0 + c];
    }
    const int nbuf = 2 * rowbytes <= fix_off ? 2 : 1;
    const int nch = max(1, min(a.m, fix_off / nbuf / rowbytes));
    const int buf_bytes = nch * rowbytes;
    __syncthreads();

    // Rows of channels [cb, cb + nch) into `dat`: wave w stages rows w, w + 4,
    // ..., whole 16-byte pieces through a raw buffer resource sized to the
    // row's whole valid pieces (zeros past them); the piece that straddles the
    // row's end, if any, byte by byte.
    auto stage = [&](int cb, uint8_t* dat) {
        const int nc = min(nch, a.m - cb);
        for (int c = wave; c < nc; c += kWaves) {
            const int64_t start = static_cast<int64_t>(u0) + uniform(st0[cb + c]);
            int64_t nb64 = a.x_len - start;                     // valid bytes of the staged row
            nb64 = nb64 < 0 ? 0 : (nb64 > rowbytes ? rowbytes : nb64);
            const int nb = uniform(static_cast<int>(nb64));
            const int part = (nb & 15) ? nb >> 4 : -1;
            const uint8_t* row = a.x + static_cast<size_t>(ch0 + cb + c) * a.x_pitch + start;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<uint8_t*>(row), static_cast<short>(0), nb & ~15, kRawBufferWord3);
            uint8_t* dst = dat + c * rowbytes;
            const int kfull = W >> 8;
            for (int k = 0; k < kfull; ++k)
                if (lane + 64 * k != part)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, to_lds(dst + 1024 * k), 16, 16 * lane + 1024 * k, 0,
                                                             0, 0);
            {
                const int i = lane + 64 * kfull;
                if (4 * i < W && i != part)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, to_lds(dst + 1024 * kfull), 16, 16 * i, 0, 0, 0);
            }
            if (part >= 0 && (part & 63) == lane) {
                const TX_GLOBAL uint8_t* src = to_global(row) + 16 * part;
                uint32_t d[4] = {0u, 0u, 0u, 0u};
                for (int b = 0; b < (nb & 15); ++b) d[b >> 2] |= static_cast<uint32_t>(src[b]) << (8 * (b & 3));
                *reinterpret_cast<uint4*>(dst + 16 * part) = make_uint4(d[0], d[1], d[2], d[3]);
            }
        }
    };

    float acc[JW][4 * Q];
#pragma unroll
    for (int jj = 0; jj < JW; ++jj)
#pragma unroll
        for (int q = 0; q < 4 * Q; ++q) acc[jj][q] = 0.0f;
    const int lane_b = 4 * Q * lane;                               // byte offset of the lane's first dword

    stage(0, lds);
    for (int cb = 0, r = 0; cb < a.m; cb += nch, ++r) {
        const int nc = min(nch, a.m - cb);
        const uint8_t* dat = lds + (r & (nbuf - 1)) * buf_bytes;
        // This wave's rows of the round have landed; after the barrier every
        // wave's have, and nobody still reads the other buffer.
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        __syncthreads();
        if (nbuf == 2 && cb + nch < a.m) stage(cb + nch, lds + ((r + 1) & 1) * buf_bytes);
        const int32_t* tw = tab + cb * J + wave * JW;
        for (int c = 0; c < nc; ++c) {
            const float sc = wsc[cb + c];                          // one address: a broadcast read
            const float of = wof[cb + c];
#pragma unroll
            for (int jj = 0; jj < JW; ++jj) {
                const int e = uniform(tw[c * J + jj]) + c * rowbytes;
                const uint32_t k = static_cast<uint32_t>(e & 3);
                const uint32_t* p = reinterpret_cast<const uint32_t*>(dat + (e & ~3) + lane_b);
                uint32_t w[Q + 1];
#pragma unroll
                for (int q = 0; q <= Q; ++q) w[q] = p[q];
                // the channel's normalised sample, rounded once, then added
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const uint32_t v = align_b32(w[q + 1], w[q], k);
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[jj][4 * q + b] += __builtin_fmaf(byte_f(v, b), sc, of);
                }
            }
        }
        if (nbuf == 1 && cb + nch < a.m) {
            __syncthreads();
            stage(cb + nch, lds);
        }
    }
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) {
        const int j = j0 + wave * JW + jj;
        if (j <= jl) {
            TX_GLOBAL float* out = to_global(a.B) + (static_cast<size_t>(j) * a.nsub + s) * a.B_pitch + u0 + 4 * Q * lane;
#pragma unroll
            for (int q = 0; q < Q; ++q)
                *reinterpret_cast<TX_GLOBAL float4*>(out + 4 * q) =
                    make_float4(acc[jj][4 * q], acc[jj][4 * q + 1], acc[jj][4 * q + 2], acc[jj][4 * q + 3]);
        }
    }
}

// ---------------------------------------------------------------------------
// Stage 2.  Workgroup = (group j, up to kNormIW of its trials, TT = 768
// outputs): lane l of wave w owns the 3 consecutive outputs from
// 3 (64 w + l), so its words of a (sub-band, trial) are one paired and one
// single 4-byte read from one base (3 is odd: the lanes' addresses fall in
// distinct banks).  Sub-band rows are staged, a round at a time, as floats
// from the first trial's shift rounded down to 4 floats, with loads straight
// into LDS (16-byte pieces), double-buffered where two rounds fit; every
// output adds its sub-bands in order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void stage2_norm_kernel(Stage2NormArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr int IW = kNormIW;
    constexpr int TT = kNormTT2;
    const int tile = xcd_tile(static_cast<int>(blockIdx.x), a.ngroups * a.n_ichunks * a.n_ttiles);
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
    const int lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const TX_GLOBAL int32_t* __restrict__ rT = to_global(a.rT);
    const size_t dp = static_cast<size_t>(a.dpad);
    int* red = reinterpret_cast<int*>(lds);

    int sp = 0;
    for (int s = tid; s < a.nsub; s += kThreads) {
        const TX_GLOBAL int32_t* r = rT + static_cast<size_t>(s) * dp;
        sp = max(sp, r[il] - (r[i0] & ~3));
    }
    sp = uniform(block_max(sp, red));
    const int rowf = (sp + TT + 3) & ~3;                  // staged floats per row
    const int tab_off = (a.lds_bytes - ((IW * a.nsub * 4 + 15) & ~15)) & ~15;
    int32_t* tab = reinterpret_cast<int32_t*>(lds + tab_off);   // [nsub][IW]: shift from the staged start
    for (int t = tid; t < IW * a.nsub; t += kThreads) {
        const int s = t / IW, k = t - s * IW;
        const TX_GLOBAL int32_t* r = rT + static_cast<size_t>(s) * dp;
        tab[t] = r[i0 + min(k, ni - 1)] - (r[i0] & ~3);
    }
    const int rowb = 4 * rowf;
    const int nbuf = 2 * 4 * rowb <= tab_off ? 2 : 1;     // two rounds of at least 4 rows, or one buffer
    const int nsb = max(1, min(a.nsub, tab_off / (nbuf * rowb)));
    const int buf_bytes = nsb * rowb;
    __syncthreads();

    const TX_GLOBAL float* Bj = to_global(a.B) + static_cast<size_t>(j) * a.nsub * a.B_pitch;
    // Rows [sb, sb + nsb) into `dat`: wave w stages rows w, w + 4, ...
    auto stage = [&](int sb, uint8_t* dat) {
        const int ns = min(nsb, a.nsub - sb);
        for (int r = wave; r < ns; r += kWaves) {
            const int s = sb + r;
            const TX_GLOBAL float* src = Bj + static_cast<size_t>(s) * a.B_pitch + t0 + (rT[static_cast<size_t>(s) * dp + i0] & ~3);
            uint8_t* dst = dat + r * rowb;
            for (int k = 0; 256 * k < rowf; ++k) {
                const int i = lane + 64 * k;              // 16-byte piece (4 floats) of the row
                if (4 * i < rowf)
                    __builtin_amdgcn_global_load_lds(reinterpret_cast<const TX_GLOBAL void*>(src + 4 * i),
                                                     to_lds(dst + 1024 * k), 16, 0, 0);
            }
        }
    };

    float acc[IW][3];
#pragma unroll
    for (int k = 0; k < IW; ++k)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[k][q] = 0.0f;
    const int lo = 3 * (64 * wave + lane);                         // the lane's first output
    stage(0, lds);
    for (int sb = 0, rd = 0; sb < a.nsub; sb += nsb, ++rd) {
        const int ns = min(nsb, a.nsub - sb);
        const float* rows = reinterpret_cast<const float*>(lds + (rd & (nbuf - 1)) * buf_bytes);
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        __syncthreads();
        if (nbuf == 2 && sb + nsb < a.nsub) stage(sb + nsb, lds + ((rd + 1) & 1) * buf_bytes);
        for (int r = 0; r < ns; ++r) {
            const float* row = rows + r * rowf + lo;
#pragma unroll
            for (int k0 = 0; k0 < IW; k0 += 4) {
#pragma unroll
                for (int k = k0; k < k0 + 4; ++k) {
                    const float* p = row + uniform(tab[(sb + r) * IW + k]);
#pragma unroll
                    for (int q = 0; q < 3; ++q) acc[k][q] += p[q];
                }
                // a group of 4 trials' reads at a time (registers)
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (nbuf == 1 && sb + nsb < a.nsub) {
            __syncthreads();
            stage(sb + nsb, lds);
        }
    }
#pragma unroll
    for (int k = 0; k < IW; ++k) {                      // compile-time indices: acc stays in registers
        if (k < ni) {
            TX_GLOBAL float* out = to_global(a.Y) + static_cast<size_t>(i0 + k) * a.y_pitch + t0 + lo;
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (t0 + lo + q < a.nt) out[q] = acc[k][q];
        }
    }
}

// ---------------------------------------------------------------------------
// Matched filter of float series.  One workgroup per row, which reads the row
// once, in tiles of kNormBoxTile window starts (thread tid owns the starts
// tid + 256 m):
//  * each tile's float64 running sums of its kNormBoxTile + longest-width
//    samples go to LDS; the same loads accumulate the float64 sum and sum of
//    squares of the row;
//  * for a fixed width the S/N is a non-decreasing function of the window
//    sum, so the per-width peak is found on the sums alone: every lane keeps
//    the largest sum of its starts per width, the wavefront's largest is
//    compared with the wavefront's best so far, and only when it beats it (a
//    few tiles per row) does the wavefront look up the earliest start
//    reaching it; each wavefront's largest sums per (tile, width) are kept in
//    LDS where they fit.
// Then the mean and sigma give each width's peak S/N (the largest over widths,
// ties to the smaller width), and per width S*, the least float64 sum whose
// S/N (the same float64 expression) reaches gamma, by bisection over the
// ordered doubles.  Only tiles where some wavefront's largest sum reaches S*
// are scanned again, and there the wavefront evaluates its starts' S/N at
// every width and lists those whose best reaches gamma.  NWT: widths the
// instance holds (slots past the row's widths repeat its last width).
// ---------------------------------------------------------------------------
constexpr int kNormBoxTile = 4096;
constexpr int kNormBoxPer = kNormBoxTile / kThreads;                 // starts per thread and tile
constexpr int kNormScanPer = (kNormBoxTile + TX_MAX_WIDTH) / kThreads;  // running-sum samples per thread
constexpr int kNormTmaxLds = 16 * 1024;

template <int NWT>
struct NormBoxShared {
    double wsum[kWaves];
    double red1[kWaves], red2[kWaves];
    double wm[kWaves][NWT];              // per wavefront: largest sum per width in this tile,
    double wS[kWaves][NWT];              // the largest so far, and
    int32_t wT[kWaves][NWT];             // its earliest start
    double sthr[NWT];                    // least sum reaching gamma per width (NaN: none)
    int32_t wd[NWT];
    double rs[NWT];
    double mean, inv;
    int state;
};

// Dynamic LDS: the running sums P of a tile (kNormBoxTile + longest width +
// 1 values), then (where it fits) the table [tile][NWT] of the workgroup's
// largest sum per tile and width.
extern __shared__ double tx_nbox_dyn[];

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// One step of a wavefront max of a float64: both halves moved by the same DPP
// pattern (lanes it does not write take -inf), then the larger kept.
template <int CTRL, int ROWS>
__device__ __forceinline__ double wave_max_step_d(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, static_cast<uint32_t>(b), CTRL, ROWS, 0xF, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp(0xFFF00000u, static_cast<uint32_t>(b >> 32), CTRL, ROWS, 0xF, false);
    const double o = __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
    return __builtin_fmax(v, o);
}

// Wavefront max (quad, half-row and row permutes, then the row broadcasts of
// 15 and 31), read from lane 63.  No operand is NaN.
__device__ __forceinline__ double wave_max_d(double v) {
    v = wave_max_step_d<0xB1, 0xF>(v);
    v = wave_max_step_d<0x4E, 0xF>(v);
    v = wave_max_step_d<0x141, 0xF>(v);
    v = wave_max_step_d<0x140, 0xF>(v);
    v = wave_max_step_d<0x142, 0xA>(v);
    v = wave_max_step_d<0x143, 0xC>(v);
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(b)), 63);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(b >> 32)), 63);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ __forceinline__ int32_t wave_min_i32_n(int32_t v) {
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0xB1, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x4E, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x141, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x140, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x142, 0xA, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x143, 0xC, 0xF, false));
    return __builtin_amdgcn_readlane(v, 63);
}

// S/N of a window sum (the one expression used for peaks, candidates and S*).
__device__ __forceinline__ double snr_f(double S, int w, double mean, double inv, double rsw) {
    return ((S - static_cast<double>(w) * mean) * inv) * rsw;
}

// Doubles in a signed 64-bit order (for non-NaN values): the bits for
// non-negative ones, the magnitude bits flipped for negative ones.  The map
// is its own inverse.
__device__ __forceinline__ int64_t dbl_key(int64_t bits) { return bits ^ ((bits >> 63) & INT64_MAX); }

// Least double S in [-inf, +inf] with snr_f(S) >= gamma (snr_f does not
// decrease with S: inv and rsw are positive); NaN when none reaches it.
__device__ __forceinline__ double least_sum_reaching(double gamma, int w, double mean, double inv, double rsw) {
    const double ninf = -__builtin_inf(), pinf = __builtin_inf();
    if (snr_f(ninf, w, mean, inv, rsw) >= gamma) return ninf;
    if (!(snr_f(pinf, w, mean, inv, rsw) >= gamma)) return __builtin_nan("");
    int64_t lo = dbl_key(__builtin_bit_cast(int64_t, ninf));    // fails
    int64_t hi = dbl_key(__builtin_bit_cast(int64_t, pinf));    // passes
    while (static_cast<uint64_t>(hi) - static_cast<uint64_t>(lo) > 1u) {
        const int64_t mid = static_cast<int64_t>(static_cast<uint64_t>(lo) +
                                                 (static_cast<uint64_t>(hi) - static_cast<uint64_t>(lo)) / 2u);
        if (snr_f(__builtin_bit_cast(double, dbl_key(mid)), w, mean, inv, rsw) >= gamma) hi = mid; else lo = mid;
    }
    return __builtin_bit_cast(double, dbl_key(hi));
}

// Float64 running sums P[e] = sum of y[t0 .. t0 + e) for e <= L (zeros past
// T): each thread sums kNormScanPer consecutive samples; a wavefront scan and
// the earlier wavefronts' totals give its base.  COUNT: add the tile's own
// samples (e < kNormBoxTile) to the sum and sum of squares.
template <bool COUNT, int NWT>
__device__ __forceinline__ void norm_scan_tile(const TX_GLOBAL float* __restrict__ y, int T, int t0, int L, bool vec,
                                               NormBoxShared<NWT>& sh, int tid, double& m1, double& m2) {
    constexpr int kPer = kNormScanPer;
    const int lane = tid & 63, wave = tid >> 6;
    const int e0 = kPer * tid;
    const int64_t tb = static_cast<int64_t>(t0) + e0;
    double v[kPer];
    if (vec && e0 + kPer <= L && tb + kPer <= T) {
#pragma unroll
        for (int k = 0; k < kPer / 4; ++k) {
            const float4 q = *reinterpret_cast<const TX_GLOBAL float4*>(y + tb + 4 * k);
            v[4 * k] = q.x;
            v[4 * k + 1] = q.y;
            v[4 * k + 2] = q.z;
            v[4 * k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kPer; ++k) v[k] = (e0 + k < L && tb + k < T) ? static_cast<double>(y[tb + k]) : 0.0;
    }
    if (COUNT) {
        const int own = kNormBoxTile - e0;           // samples of this tile (the rest belong to the next)
        double a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const double x = k < own ? v[k] : 0.0;
            a1 += x;
            a2 += x * x;
        }
        m1 += a1;
        m2 += a2;
    }
    double run = 0.0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) run += v[k];
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
        if (e0 + k <= L) tx_nbox_dyn[e0 + k] = base;
        base += v[k];
    }
    __syncthreads();
}

// Per-width largest sums of one tile (each wavefront's in sh.wm) and the
// wavefront bests.  TAIL: some windows reach past the row end (they count as
// -inf).
template <int NWT, bool TAIL>
__device__ __forceinline__ void norm_peak_tile(NormBoxShared<NWT>& sh, int T, int t0, int tid) {
    const int wave = tid >> 6;
    double Pt[kNormBoxPer];
#pragma unroll
    for (int j = 0; j < kNormBoxPer; ++j) Pt[j] = tx_nbox_dyn[tid + 256 * j];
    double tm[NWT];
#pragma unroll
    for (int i = 0; i < NWT; ++i) {
        const int w = sh.wd[i];
        const double* p = tx_nbox_dyn + tid + w;
        double m = -__builtin_inf();
#pragma unroll
        for (int j = 0; j < kNormBoxPer; ++j) {
            double S = p[256 * j] - Pt[j];
            if (TAIL) S = t0 + tid + 256 * j + w <= T ? S : -__builtin_inf();
            m = __builtin_fmax(m, S);
        }
        tm[i] = m;
        // Keep each width's LDS reads next to their arithmetic.
        __builtin_amdgcn_sched_barrier(0);
    }
    // Wavefront maxima (independent reductions, interleaved), left in LDS
    // for the rolled loop below to read by width.
    double wm[NWT];
#pragma unroll
    for (int i = 0; i < NWT; ++i) wm[i] = wave_max_d(tm[i]);
    if ((tid & 63) == 0) {
#pragma unroll
        for (int i = 0; i < NWT; ++i) sh.wm[wave][i] = wm[i];
    }
#pragma unroll 1
    for (int ii = 0; ii < NWT; ++ii) {
        const double m = sh.wm[wave][ii];
        if (m > sh.wS[wave][ii]) {                      // wavefront-uniform, a few tiles per row
            const int w = sh.wd[ii];
            int32_t first = INT32_MAX;
#pragma unroll 1
            for (int j = kNormBoxPer - 1; j >= 0; --j) {   // rolled: this path is rare
                const int e = tid + 256 * j;
                const int t = t0 + e;
                const double S = tx_nbox_dyn[e + w] - tx_nbox_dyn[e];
                first = ((!TAIL || t + w <= T) && S == m) ? t : first;
            }
            const int32_t ft = wave_min_i32_n(first);
            if ((tid & 63) == 0) {
                sh.wS[wave][ii] = m;
                sh.wT[wave][ii] = ft;
            }
        }
    }
}

// A wavefront's candidates in one tile: every start whose best S/N over the
// widths (ties to the smaller width) reaches gamma.
template <int NWT>
__device__ __forceinline__ void norm_cand_wave(const BoxcarNormArgs& a, NormBoxShared<NWT>& sh, int row, int t0, double mean,
                                               double inv, int tid) {
    const int T = a.nt;
#pragma unroll 1
    for (int j = 0; j < kNormBoxPer; ++j) {
        const int e = tid + 256 * j;
        const int t = t0 + e;
        if (t >= T) break;
        const double pe = tx_nbox_dyn[e];
        double best = -__builtin_inf();
        int bw = -1;
        for (int i = 0; i < a.ne; ++i) {
            const int w = sh.wd[i];
            if (t + w > T) continue;
            const double sn = snr_f(tx_nbox_dyn[e + w] - pe, w, mean, inv, sh.rs[i]);
            if (bw < 0 || sn > best) {
                best = sn;
                bw = w;
            }
        }
        if (bw > 0 && best >= a.gamma) {
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
}

template <int NWT>
__global__ __launch_bounds__(kThreads) void boxcar_norm_kernel(BoxcarNormArgs a) {
    __shared__ NormBoxShared<NWT> sh;
    const int row = static_cast<int>(blockIdx.x);
    if (row >= a.ndm) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int T = a.nt;
    const TX_GLOBAL float* __restrict__ y = to_global(a.y) + static_cast<size_t>(row) * a.pitch;
    const bool vec = ((reinterpret_cast<uintptr_t>(a.y) + static_cast<uintptr_t>(row) * a.pitch * 4) & 15) == 0;
    const bool keep_tmax = a.tmax_ok != 0;
    const int L = kNormBoxTile + a.wmax;
    double* tmax = tx_nbox_dyn + ((L + 2) & ~1);
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
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NWT; ++i) {
            sh.wS[wave][i] = -__builtin_inf();
            sh.wT[wave][i] = 0;
        }
    }
    // (the first tile's barriers order these writes before their reads)

    const int ntiles = (T + kNormBoxTile - 1) / kNormBoxTile;
    double m1 = 0.0, m2 = 0.0;
    for (int tile = 0; tile < ntiles; ++tile) {
        const int t0 = tile * kNormBoxTile;
        // The thread index, opaque to the compiler in every tile: else it
        // hoists lane-dependent addresses out of this loop.
        int tv = tid;
        asm volatile("" : "+v"(tv));
        norm_scan_tile<true, NWT>(y, T, t0, L, vec, sh, tv, m1, m2);
        if (a.ne > 0) {
            if (t0 + kNormBoxTile + a.wmax > T) norm_peak_tile<NWT, true>(sh, T, t0, tv);
            else norm_peak_tile<NWT, false>(sh, T, t0, tv);
        }
        __syncthreads();
        // The workgroup's largest sum per width of this tile (the next tile's
        // barriers order this before sh.wm is written again).
        if (keep_tmax && tid < NWT)
            tmax[tile * NWT + tid] = __builtin_fmax(__builtin_fmax(sh.wm[0][tid], sh.wm[1][tid]),
                                                    __builtin_fmax(sh.wm[2][tid], sh.wm[3][tid]));
    }

    // Statistics.
    m1 = wave_sum_d(m1);
    m2 = wave_sum_d(m2);
    if (lane == 0) {
        sh.red1[wave] = m1;
        sh.red2[wave] = m2;
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

    // The row's peak: per width the largest sum over the wavefronts (earliest
    // start on ties) and its S/N; the largest S/N over widths, ties to the
    // smaller width.
    if (tid == 0 && a.want_peaks) {
        double best = 0.0;
        int bw = -1;
        int64_t btm = 0;
        for (int i = 0; i < a.ne; ++i) {
            double S = sh.wS[0][i];
            int32_t t = sh.wT[0][i];
            for (int w2 = 1; w2 < kWaves; ++w2)
                if (sh.wS[w2][i] > S || (sh.wS[w2][i] == S && sh.wT[w2][i] < t)) {
                    S = sh.wS[w2][i];
                    t = sh.wT[w2][i];
                }
            if (S == -__builtin_inf()) continue;
            const double s = snr_f(S, sh.wd[i], mean, inv, sh.rs[i]);
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

    // Candidates: only tiles whose largest sum reaches some width's S*; every
    // tile where the table did not fit.
    if (a.want_cands && a.ne > 0) {
        if (tid < a.ne) sh.sthr[tid] = least_sum_reaching(a.gamma, sh.wd[tid], mean, inv, sh.rs[tid]);
        __syncthreads();
        for (int tile = 0; tile < ntiles; ++tile) {
            bool hit = !keep_tmax;
            if (keep_tmax)
                for (int i = 0; i < a.ne; ++i) hit = hit || tmax[tile * NWT + i] >= sh.sthr[i];
            if (!hit) continue;                           // workgroup-uniform
            const int t0 = tile * kNormBoxTile;
            double u1 = 0.0, u2 = 0.0;
            norm_scan_tile<false, NWT>(y, T, t0, L, vec, sh, tid, u1, u2);
            norm_cand_wave(a, sh, row, t0, mean, inv, tid);
            __syncthreads();
        }
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
    g.n_jchunks = (p->ngroups + 4 * kNormJW - 1) / (4 * kNormJW);
    // stage 2 stages floats [start, start + rowf) of a series, start <= last
    // tile start + max extent; rowf <= spread + TT + 3
    const int sp2 = plan_spread2(p, kNormIW) + 3;
    const int64_t need = static_cast<int64_t>(std::max(g.n_ttiles2 - 1, 0)) * kNormTT2 + p->max_extent + sp2 + kNormTT2 + 4;
    const int tt1 = 256 * kNormQ;
    g.B_pitch = (std::max<int64_t>(need, nt + p->max_extent) + tt1 - 1) / tt1 * tt1;
    g.n_ttiles1 = static_cast<int32_t>(g.B_pitch / tt1);
    g.ws_bytes = (static_cast<int64_t>(p->ngroups) * p->nsub * g.B_pitch * 4 + 255) / 256 * 256;
    const int sp1 = plan_spread1(p, 4 * kNormJW) + 15;
    const int row1 = 4 * (((sp1 >> 2) + 64 * kNormQ + 1 + 3) & ~3);   // a staged row (as the kernel sizes it)
    g.lds1 = std::max(kNormLds1, row1 + ((p->m * (4 * kNormJW + 3) * 4 + 15) & ~15) + 64);
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
    // Dynamic LDS: the running sums (sized by the longest width), then the
    // workgroup's largest sum per (tile, width) where it fits in
    // kNormTmaxLds; otherwise candidates rescan every tile.
    BoxcarNormArgs b = a;
    const int nwt = boxcar_nwt(a.ne);
    const int pbytes = ((kNormBoxTile + a.wmax + 2) & ~1) * 8;
    const int64_t tbytes = static_cast<int64_t>((a.nt + kNormBoxTile - 1) / kNormBoxTile) * nwt * 8;
    b.tmax_ok = tbytes <= kNormTmaxLds ? 1 : 0;
    const int lds = pbytes + (b.tmax_ok ? static_cast<int>(tbytes) : 0);
    const int prof = prof_begin(TX_KERNEL_BOXCAR, stream);
    switch (nwt) {
        case 4: hipLaunchKernelGGL(boxcar_norm_kernel<4>, dim3(a.ndm), dim3(kThreads), lds, stream, b); break;
        case 8: hipLaunchKernelGGL(boxcar_norm_kernel<8>, dim3(a.ndm), dim3(kThreads), lds, stream, b); break;
        case 10: hipLaunchKernelGGL(boxcar_norm_kernel<10>, dim3(a.ndm), dim3(kThreads), lds, stream, b); break;
        case 12: hipLaunchKernelGGL(boxcar_norm_kernel<12>, dim3(a.ndm), dim3(kThreads), lds, stream, b); break;
        case 16: hipLaunchKernelGGL(boxcar_norm_kernel<16>, dim3(a.ndm), dim3(kThreads), lds, stream, b); break;
        default: hipLaunchKernelGGL(boxcar_norm_kernel<32>, dim3(a.ndm), dim3(kThreads), lds, stream, b); break;
    }
    const hipError_t e = hipGetLastError();
    prof_end(prof, stream);
    return e;
}

}  // namespace tx
