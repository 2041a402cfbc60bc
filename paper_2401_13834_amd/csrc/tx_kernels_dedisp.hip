// Two-stage sub-band dedispersion kernels for gfx950 (MI355X).
//
// Layout: filterbank rows are channel-major uint8; first-stage series are
// uint16 [group][sub-band][time]; the output is int32 [trial][time].  All sums
// are integer and exact, so any tiling gives bit-identical results.
//
// Both stages are shift-and-add with one shift per (trial, row) that is the
// same for every lane of a wave: lanes walk the time axis and read one
// contiguous LDS window per (trial, row).  A per-(row, trial) table gives the
// word to read and the remaining byte (stage 1) or copy (stage 2) of the
// shift.  Stage 1 keeps one copy of a row and joins neighbouring dwords with
// v_alignbyte; stage 2 keeps two copies, one element apart, and reads whole
// dwords.  Lane address patterns are chosen so that the 4-byte and paired
// 4-byte LDS reads are bank-conflict free.
#include <algorithm>
#include <type_traits>

#include "tx_internal.h"

namespace tx {

__device__ __forceinline__ uint32_t perm_b32(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint64_t>(v)), l);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint64_t>(v) >> 32), l);
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}



// A wavefront's own LDS span: its LDS operations complete in order, so its
// later reads see its earlier writes; the fence keeps the compiler from moving
// them across each other.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Stage 1: B[j][s][u] = sum over ch in s of x[ch][u + D(c_j, f_ch)].
//
// Workgroup = (sub-band s, J = 4*JW coarse trials, TT = 256*Q outputs); wave w
// owns trials j0 + w*JW .. + JW-1 and lane l owns the Q consecutive output
// dwords Q l .. Q l + Q - 1 (4 outputs each).  A lane reads its Q + 1 input
// dwords of a (channel, trial) as (Q + 1) / 2 paired 4-byte reads from one
// base; Q is odd, so the lanes' addresses (Q dwords apart) fall in distinct
// banks.  That is 1 + 1/Q dwords of LDS read per output dword, against 2 when
// a lane reads words w and w + 1 of every output dword separately.  Channel
// rows are staged starting at the row's shift for the first trial, rounded
// down to 16 bytes, with buffer loads straight into LDS, double-buffered so
// that a round of rows loads while the previous one is summed; a
// per-(channel, trial) table, built once per workgroup, holds the byte
// offset of the first word and the remaining byte shift k.  v_alignbyte picks
// the 4 input bytes of an output dword, a byte permute picks bytes 1 and 3
// into 16-bit lanes.
//
// "full" accumulates the 4 bytes as one 32-bit word (carries cross bytes) and
// "odd" accumulates bytes 1 and 3 as two 16-bit lanes; at the end
// full - (odd << 8) = (sum b0) | (sum b2) << 16 exactly, because every 16-bit
// sum of <= 256 bytes is < 2^16.  Channels are taken in pairs so that two
// contributions and the accumulator meet in one 3-input add.
// ---------------------------------------------------------------------------
template <int Q, int JW>
__device__ __forceinline__ void stage1_tile(const Stage1Args& a, int tile, uint8_t* lds, int* red, int tid) {
    constexpr int J = JW * kWaves;
    constexpr int TT = 256 * Q;
    constexpr uint32_t kOdd = 0x0C030C01u;   // bytes 1 and 3 into 16-bit lanes
    const int jc = tile % a.n_jchunks;
    const int rest = tile / a.n_jchunks;
    const int tt = rest % a.n_ttiles;
    const int s = rest / a.n_ttiles;
    const int j0 = jc * J;
    const int jl = min(j0 + J, a.ngroups) - 1;
    const int u0 = tt * TT;
    const int lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const int ch0 = s * a.m;
    const TX_GLOBAL int32_t* __restrict__ dT = to_global(a.dT);
    const size_t gp = static_cast<size_t>(a.gpad);

    // Every row starts at byte x_off of its 16-byte aligned base, so shifts
    // are D + x_off from the base.  Largest shift (from the 16-byte aligned
    // staging start) in this workgroup:
    const int xo = a.x_off;
    int sp = 0;
    for (int c = tid; c < a.m; c += kThreads) {
        const TX_GLOBAL int32_t* r = dT + static_cast<size_t>(ch0 + c) * gp;
        sp = max(sp, (r[jl] + xo) - ((r[j0] + xo) & ~15));
    }
    sp = uniform(block_max(sp, red));
    const int W = ((sp >> 2) + 64 * Q + 1 + 3) & ~3;      // dwords per staged row
    const int rowbytes = 4 * W;

    // The workgroup's tables, built once at the top of LDS: per channel its
    // staging start (16-byte aligned, from the row's base; complemented for a
    // dropped channel) and per (channel, trial) the shift from that start.
    // Staging rounds then read only LDS and never wait on global memory.
    const int fix_off = (a.lds_bytes - ((a.m * (J + 1) * 4 + 15) & ~15)) & ~15;
    int32_t* tabA = reinterpret_cast<int32_t*>(lds + fix_off);   // [m][J]
    int32_t* rst = tabA + a.m * J;                                // [m]
    for (int t = tid; t < a.m * J; t += kThreads) {
        const int c = t / J, k = t - c * J;
        const TX_GLOBAL int32_t* r = dT + static_cast<size_t>(ch0 + c) * gp;
        tabA[t] = (r[min(j0 + k, jl)] + xo) - ((r[j0] + xo) & ~15);
    }
    for (int c = tid; c < a.m; c += kThreads) {
        const int ch = ch0 + c;
        const int st = (dT[static_cast<size_t>(ch) * gp + j0] + xo) & ~15;
        const bool keep = !a.mask || to_global(a.mask)[ch] != 0;   // a dropped channel is staged as zeros
        rst[c] = keep ? st : ~st;
    }
    // Two staging buffers where two rows fit below the tables: round r + 1's
    // rows load while round r is summed.  Otherwise one, staged between two
    // barriers.
    const int nbuf = 2 * rowbytes <= fix_off ? 2 : 1;
    const int nch = max(1, min(a.m, fix_off / nbuf / rowbytes));
    const int buf_bytes = nch * rowbytes;
    __syncthreads();

    // Stage the rows of channels [cb, cb + nch) into `dat`.  Whole 16-byte
    // pieces go from global memory straight to LDS (buffer_load ... lds: no
    // registers, completes in the background; a wave's 64 pieces land at
    // consecutive 16-byte slots of one 1 KB span).  Each row is read through
    // a raw buffer resource sized to the row's whole valid pieces, so the
    // hardware range check returns zeros for the pieces past the row's end,
    // and for a dropped channel (size 0) everywhere.  The one piece that
    // straddles the end goes through registers, byte by byte, with zeros past
    // the end (nothing past the row's valid bytes is read).
    auto stage = [&](int cb, uint8_t* dat) {
        const int nc = min(nch, a.m - cb);
        for (int c = wave; c < nc; c += kWaves) {
            const int v = uniform(rst[cb + c]);
            const int64_t start = static_cast<int64_t>(u0) + (v >= 0 ? v : ~v);
            int64_t nb64 = v >= 0 ? a.x_len + xo - start : 0;   // valid bytes of the staged row
            nb64 = nb64 < 0 ? 0 : (nb64 > rowbytes ? rowbytes : nb64);
            const int nb = uniform(static_cast<int>(nb64));
            const int part = (nb & 15) ? nb >> 4 : -1;         // the straddling piece, if any
            const uint8_t* row = a.x + static_cast<size_t>(ch0 + cb + c) * a.x_pitch + start;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<uint8_t*>(row), static_cast<short>(0), nb & ~15, kRawBufferWord3);
            uint8_t* dst = dat + c * rowbytes;
            // Piece i = lane + 64 k of the row.  Whole spans of 64 pieces, then
            // the last partial span; the straddling piece is skipped only where
            // the row has one (uniform branch).
            const int kfull = W >> 8;
            if (part < 0) {
                for (int k = 0; k < kfull; ++k)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, to_lds(dst + 1024 * k), 16, 16 * lane + 1024 * k, 0,
                                                             0, 0);
            } else {
                for (int k = 0; k < kfull; ++k)
                    if (lane + 64 * k != part)
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, to_lds(dst + 1024 * k), 16, 16 * lane + 1024 * k,
                                                                 0, 0, 0);
            }
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

    uint32_t full[JW][Q], odd[JW][Q];
#pragma unroll
    for (int jj = 0; jj < JW; ++jj)
#pragma unroll
        for (int q = 0; q < Q; ++q) full[jj][q] = odd[jj][q] = 0u;

    stage(0, lds);
    for (int cb = 0, r = 0; cb < a.m; cb += nch, ++r) {
        const int nc = min(nch, a.m - cb);
        const uint8_t* dat = lds + (r & (nbuf - 1)) * buf_bytes;
        // This wave's background loads into `dat` are done; after the barrier
        // every wave's are, and nobody still reads the other buffer.
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        __syncthreads();
        if (nbuf == 2 && cb + nch < a.m) stage(cb + nch, lds + ((r + 1) & 1) * buf_bytes);
        const int32_t* tw = tabA + cb * J + wave * JW;
        const int lane_b = 4 * Q * lane;   // byte offset of the lane's first dword
        int c = 0;
        for (; c + 1 < nc; c += 2) {
#pragma unroll
            for (int jj = 0; jj < JW; ++jj) {
                const int e0 = uniform(tw[c * J + jj]) + c * rowbytes;
                const int e1 = uniform(tw[(c + 1) * J + jj]) + (c + 1) * rowbytes;
                const uint32_t k0 = static_cast<uint32_t>(e0 & 3), k1 = static_cast<uint32_t>(e1 & 3);
                const uint32_t sel0 = kOdd + k0 * 0x00010001u, sel1 = kOdd + k1 * 0x00010001u;
                const uint32_t* p0 = reinterpret_cast<const uint32_t*>(dat + (e0 & ~3) + lane_b);
                const uint32_t* p1 = reinterpret_cast<const uint32_t*>(dat + (e1 & ~3) + lane_b);
                uint32_t a[Q + 1], b[Q + 1];
#pragma unroll
                for (int q = 0; q <= Q; ++q) {
                    a[q] = p0[q];
                    b[q] = p1[q];
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    full[jj][q] += align_b32(a[q + 1], a[q], k0) + align_b32(b[q + 1], b[q], k1);
                    odd[jj][q] += perm_b32(a[q + 1], a[q], sel0) + perm_b32(b[q + 1], b[q], sel1);
                }
            }
        }
        if (c < nc) {
#pragma unroll
            for (int jj = 0; jj < JW; ++jj) {
                const int e0 = uniform(tw[c * J + jj]) + c * rowbytes;
                const uint32_t k0 = static_cast<uint32_t>(e0 & 3);
                const uint32_t sel0 = kOdd + k0 * 0x00010001u;
                const uint32_t* p0 = reinterpret_cast<const uint32_t*>(dat + (e0 & ~3) + lane_b);
                uint32_t a[Q + 1];
#pragma unroll
                for (int q = 0; q <= Q; ++q) a[q] = p0[q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    full[jj][q] += align_b32(a[q + 1], a[q], k0);
                    odd[jj][q] += perm_b32(a[q + 1], a[q], sel0);
                }
            }
        }
        if (nbuf == 1 && cb + nch < a.m) {
            __syncthreads();
            stage(cb + nch, lds);
        }
    }

    // Outputs: a lane's Q output dwords are consecutive, so it would store
    // 8 bytes at a stride of 8 Q bytes.  Each wave passes a trial's sums
    // through its own LDS span instead, and stores them as whole contiguous
    // 512-byte runs.
    uint8_t* wb = lds + wave * (512 * Q);
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) {
        const int j = j0 + wave * JW + jj;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const uint32_t even = full[jj][q] - (odd[jj][q] << 8);
            const uint32_t w01 = perm_b32(odd[jj][q], even, 0x05040100u);
            const uint32_t w23 = perm_b32(odd[jj][q], even, 0x07060302u);
            *reinterpret_cast<uint2*>(wb + 8 * (Q * lane + q)) = make_uint2(w01, w23);
        }
        wave_lds_sync();
        if (j <= jl) {
            TX_GLOBAL uint16_t* out = to_global(a.B) + (static_cast<size_t>(j) * a.nsub + s) * a.B_pitch + u0;
#pragma unroll
            for (int q = 0; q < Q; ++q)
                *reinterpret_cast<TX_GLOBAL uint2*>(out + 4 * (lane + 64 * q)) =
                    *reinterpret_cast<const uint2*>(wb + 8 * (lane + 64 * q));
        }
        wave_lds_sync();
    }
}

// ---------------------------------------------------------------------------
// Stage 2: Y[i][t] = sum over s of B[j][s][t + rel(i, s)],
// rel(i, s) = D(dm_i, f_s) - D(c_j, f_s).
//
// Workgroup = (group j, IW of its fine trials, TT = 512*Q outputs); the 4
// waves split the time tile and each handles all IW trials.  Lane l of wave w
// owns the Q consecutive output dwords (two uint16 outputs each) from
// w*64*Q + Q l, so one address add per (sub-band, trial) serves Q reads, which
// pair into 8-byte reads; Q is odd, so the lanes' addresses fall in distinct
// banks.  Sub-band rows are staged, a round of them at a time, from the
// chunk's first trial's shift rounded down to 8 elements, twice: as they are
// and one element later, so that an even element shift reads whole dwords of
// the first copy and an odd one whole dwords of the second (one aligned 4-byte
// read per output dword, no byte joins).  The first copy loads straight from
// global memory into LDS; each wave then builds the second copy of its own
// rows from it.  A per-(trial, sub-band) table, built once per workgroup,
// holds the byte offset of the trial's first dword.  Outputs are summed as
// packed 16-bit lanes of one 32-bit word over groups of up to 4 sub-bands
// (exact while the group is at most `flush` = floor(65535 / (255 m))
// sub-bands), and each group's sum is widened into two 32-bit totals; the
// trials of a group are software-pipelined (the next trial's words are read
// while the current one is summed).
// ---------------------------------------------------------------------------
template <int IW, int Q>
__device__ __forceinline__ void stage2_tile(const Stage2Args& a, int tile, uint8_t* lds, int* red, int tid) {
    constexpr int IWP = (IW + 3) & ~3;
    constexpr int TT = 512 * Q;
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
    const int lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const TX_GLOBAL int32_t* __restrict__ rT = to_global(a.rT);
    const size_t dp = static_cast<size_t>(a.dpad);

    int sp = 0;
    for (int s = tid; s < a.nsub; s += kThreads) {
        const TX_GLOBAL int32_t* r = rT + static_cast<size_t>(s) * dp;
        sp = max(sp, r[il] - (r[i0] & ~7));
    }
    sp = uniform(block_max(sp, red));
    // A staged row is kept twice: copy 0 from the 8-element aligned start,
    // copy 1 one element later, so that every trial's window starts at a
    // dword of one of them (one aligned 4-byte read per output dword).  Copy 1
    // spans the W dwords the trials read; copy 0 holds one more 16-byte
    // piece, the next dwords copy 1 is built from.
    const int W = ((sp >> 1) + 256 * Q + 1 + 3) & ~3;
    const int W0 = W + 4;
    const int chb = 4 * (W0 + W);                  // bytes per staged sub-band row

    // The workgroup's table, built once at the top of LDS: per (trial,
    // sub-band) the byte offset of the trial's first dword within the row's
    // two copies.  Staging rounds then wait only on their own rows.  Trial
    // major, so that the entries of a group of 4 (2) sub-bands are one
    // aligned 16-byte (8-byte) read.
    const int nsp = (a.nsub + 3) & ~3;
    const int tab_off = (a.lds_bytes - IWP * nsp * 4) & ~15;
    int32_t* tab = reinterpret_cast<int32_t*>(lds + tab_off);   // [IWP][nsp]
    for (int t = tid; t < IWP * nsp; t += kThreads) {
        const int k = t / nsp, s = t - k * nsp;
        if (s < a.nsub) {
            const TX_GLOBAL int32_t* rr = rT + static_cast<size_t>(s) * dp;
            const int e = rr[i0 + min(k, ni - 1)] - (rr[i0] & ~7);
            tab[t] = (e & 1) * (4 * W0) + 4 * (e >> 1);   // copy (e & 1), dword e / 2
        }
    }
    // Sub-bands per staging round: a multiple of 4 (or 2) where that many
    // fit, so that every group's table entries are aligned.
    int nsb = max(1, min(a.nsub, tab_off / chb));
    nsb = nsb >= 4 ? (nsb & ~3) : (nsb >= 2 ? 2 : 1);
    uint8_t* dat = lds;

    // Exact 32-bit sums of the low and high 16-bit outputs of each dword.
    uint32_t lo[IW][Q], hi[IW][Q];
#pragma unroll
    for (int ii = 0; ii < IW; ++ii)
#pragma unroll
        for (int q = 0; q < Q; ++q) lo[ii][q] = hi[ii][q] = 0u;
    const TX_GLOBAL uint16_t* Bj = to_global(a.B) + static_cast<size_t>(j) * a.nsub * a.B_pitch;
    const int wbase = wave * 64 * Q + Q * lane;   // the lane's first output dword

    // G sub-bands of each trial summed as packed 16-bit lanes (exact while
    // G <= flush), then added to the 32-bit sums.  Software-pipelined over
    // the trials: trial ii + 1's words are read while trial ii is summed, and
    // the table entries of trial ii + 2 while those words are in flight, so
    // the one wait per trial finds its data already there.
    auto group = [&](auto gtag, int sb, int r) {
        constexpr int G = decltype(gtag)::value;
        uint32_t xc[G][Q], xn[G][Q];
        int tn[G];                                   // table entries (uniform) of the next trial to read
        auto tab_read = [&](int ii) {
            const int32_t* tp = tab + ii * nsp + sb + r;
            if constexpr (G == 4) {
                const int4 v = *reinterpret_cast<const int4*>(tp);
                tn[0] = v.x;
                tn[1] = v.y;
                tn[2] = v.z;
                tn[3] = v.w;
            } else if constexpr (G == 2) {
                const int2 v = *reinterpret_cast<const int2*>(tp);
                tn[0] = v.x;
                tn[1] = v.y;
            } else {
                tn[0] = tp[0];
            }
        };
        auto fetch = [&](uint32_t (&x)[G][Q]) {
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const uint32_t* p =
                    reinterpret_cast<const uint32_t*>(dat + uniform(tn[k]) + (r + k) * chb) + wbase;
#pragma unroll
                for (int q = 0; q < Q; ++q) x[k][q] = p[q];
            }
        };
        tab_read(0);
        fetch(xc);
        if (IW > 1) tab_read(1);
#pragma unroll
        for (int ii = 0; ii < IW; ++ii) {
            if (ii + 1 < IW) {
                fetch(xn);
                if (ii + 2 < IW) tab_read(ii + 2);
            }
            // Keep the compiler from sinking the reads below the adds.
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                uint32_t sum;
                if constexpr (G == 4) sum = (xc[0][q] + xc[1][q] + xc[2][q]) + xc[3][q];
                else if constexpr (G == 2) sum = xc[0][q] + xc[1][q];
                else sum = xc[0][q];
                lo[ii][q] += sum & 0xFFFFu;
                hi[ii][q] += sum >> 16;
            }
            __builtin_amdgcn_sched_barrier(0);
            if (ii + 1 < IW) {
#pragma unroll
                for (int k = 0; k < G; ++k)
#pragma unroll
                    for (int q = 0; q < Q; ++q) xc[k][q] = xn[k][q];
            }
        }
    };

    __syncthreads();
    for (int sb = 0; sb < a.nsub; sb += nsb) {
        const int ns = min(nsb, a.nsub - sb);
        // Copy 0 of wave w's rows (w, w + 4, ...) straight from global memory
        // into LDS (global_load_lds: whole 16-byte pieces, no registers; a
        // wave's 64 pieces land at consecutive 16-byte slots of one 1 KB
        // span), all in flight at once ...
        for (int r = wave; r < ns; r += kWaves) {
            const int s = sb + r;
            const TX_GLOBAL uint16_t* src =
                Bj + static_cast<size_t>(s) * a.B_pitch + t0 + (rT[static_cast<size_t>(s) * dp + i0] & ~7);
            uint8_t* dst = dat + r * chb;
            for (int k = 0; 256 * k < W0; ++k) {
                const int i = lane + 64 * k;
                if (4 * i < W0)
                    __builtin_amdgcn_global_load_lds(reinterpret_cast<const TX_GLOBAL void*>(src + 8 * i),
                                                     to_lds(dst + 1024 * k), 16, 0, 0);
            }
        }
        // ... then, once they have landed, copy 1 of the same rows from it.
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        asm volatile("" ::: "memory");
        for (int r = wave; r < ns; r += kWaves) {
            const uint32_t* c0 = reinterpret_cast<const uint32_t*>(dat + r * chb);
            uint32_t* c1 = reinterpret_cast<uint32_t*>(dat + r * chb) + W0;
            for (int i = lane; 4 * i < W; i += 64) {
                const uint4 v = *reinterpret_cast<const uint4*>(c0 + 4 * i);
                // The dword after this piece starts the next lane's piece:
                // take it with a wavefront shift (DPP wave_shl:1) rather than
                // a read at a 16-byte lane stride, which conflicts 4 ways in
                // the LDS banks.  The last lane of the wave and the last
                // active lane read it.
                uint32_t nx = __builtin_amdgcn_update_dpp(0u, v.x, 0x130, 0xF, 0xF, false);
                if (lane == 63 || 4 * (i + 1) >= W) nx = c0[4 * i + 4];
                *reinterpret_cast<uint4*>(c1 + 4 * i) = make_uint4(align_b32(v.y, v.x, 2), align_b32(v.z, v.y, 2),
                                                                   align_b32(v.w, v.z, 2), align_b32(nx, v.w, 2));
            }
        }
        __syncthreads();
        int r = 0;
        if (a.flush >= 4)
            for (; r + 4 <= ns; r += 4) group(std::integral_constant<int, 4>{}, sb, r);
        if (a.flush >= 2)
            for (; r + 2 <= ns; r += 2) group(std::integral_constant<int, 2>{}, sb, r);
        for (; r < ns; ++r) group(std::integral_constant<int, 1>{}, sb, r);
        __syncthreads();
    }

    // Outputs: with Q > 1 a lane's output pairs are consecutive, so its
    // stores would be 8 bytes at a stride of 8 Q bytes; each wave passes a
    // trial's sums through its own LDS span and stores contiguous runs.
    uint8_t* wb = lds + wave * (512 * Q);
#pragma unroll
    for (int ii = 0; ii < IW; ++ii) {
        if (Q > 1) {
#pragma unroll
            for (int q = 0; q < Q; ++q) *reinterpret_cast<uint2*>(wb + 8 * (Q * lane + q)) = make_uint2(lo[ii][q], hi[ii][q]);
            wave_lds_sync();
        }
        if (ii < ni) {
            TX_GLOBAL int32_t* out = to_global(a.Y) + static_cast<size_t>(i0 + ii) * a.y_pitch;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int64_t t = t0 + 2 * static_cast<int64_t>(wave * 64 * Q + lane + 64 * q);
                const uint2 v = Q > 1 ? *reinterpret_cast<const uint2*>(wb + 8 * (lane + 64 * q))
                                      : make_uint2(lo[ii][q], hi[ii][q]);
                if (t + 1 < a.nt) {
                    *reinterpret_cast<TX_GLOBAL int2*>(out + t) =
                        make_int2(static_cast<int32_t>(v.x), static_cast<int32_t>(v.y));
                } else if (t < a.nt) {
                    out[t] = static_cast<int32_t>(v.x);
                }
            }
        }
        if (Q > 1) wave_lds_sync();
    }
}

// ---------------------------------------------------------------------------
// Kernels: one job (arguments by value, one workgroup per tile), or a batch
// of jobs of one tile variant.  A batch launch is persistent: a grid sized to
// what the device holds at once, each workgroup taking tile after tile from
// work counters in device memory until they run out.  The job arguments,
// tile prefix sums, job count and counters are read from the batch's device
// table, so a captured graph can be replayed over another set of jobs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_job(const int* __restrict__ prefix, int njobs, int t) {
    int lo = 0, hi = njobs;                 // prefix[lo] <= t < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

template <int Q, int JW>
__global__ __launch_bounds__(kThreads) void stage1_kernel(Stage1Args a) {
    extern __shared__ __align__(16) uint8_t lds[];
    int* red = reinterpret_cast<int*>(lds);   // block_max scratch, used before anything is staged
    stage1_tile<Q, JW>(a, xcd_tile(blockIdx.x, a.nsub * a.n_ttiles * a.n_jchunks), lds, red, threadIdx.x);
}

// The batch form of the first stage is held to 5 waves per SIMD (102 VGPRs):
// left alone the persistent loop's larger function is scheduled for 4 in most
// variants (9 x 2: 110 VGPRs, 85 when held).  The 9 x 4 variant is left
// alone: held, it spills 11 dwords and runs slower.
#define TX_S1B_WAVES(Q, JW) __attribute__((amdgpu_waves_per_eu((Q) == 9 && (JW) == 4 ? 1 : 5)))

template <int Q, int JW>
__global__ __launch_bounds__(kThreads) TX_S1B_WAVES(Q, JW) void stage1_batch_kernel(const Stage1Args* __restrict__ jobs,
                                                                const int* __restrict__ prefix_base,
                                                                const int* __restrict__ info, uint32_t* queue) {
    extern __shared__ __align__(16) uint8_t lds[];
    int* red = reinterpret_cast<int*>(lds);
    const int njobs = info[0];
    if (njobs <= 0) return;
    const Stage1Args* cj = jobs + info[1];
    const int* prefix = prefix_base + info[2];
    for_each_claimed(prefix[njobs], queue, [&](int t) {
        const int jb = find_job(prefix, njobs, t);
        const Stage1Args a = cj[jb];
        // The thread index, opaque to the compiler in every tile: else it
        // keeps lane-dependent values of the tile body live across tiles.
        int tv = static_cast<int>(threadIdx.x);
        asm volatile("" : "+v"(tv));
        stage1_tile<Q, JW>(a, t - prefix[jb], lds, red, tv);
    });
}

// The 16-trial, 3-dword variant is held to 4 waves per SIMD (128 VGPRs): left
// alone it takes 131 and runs 3 waves; capped it keeps 3 dwords in scratch,
// reloaded once per staging round.  Other variants are left to the compiler.
#define TX_S2_WAVES(IW, Q) __attribute__((amdgpu_waves_per_eu((IW) == 16 && (Q) == 3 ? 4 : 1)))

template <int IW, int Q>
__global__ __launch_bounds__(kThreads) TX_S2_WAVES(IW, Q) void stage2_kernel(Stage2Args a) {
    extern __shared__ __align__(16) uint8_t lds[];
    int* red = reinterpret_cast<int*>(lds);   // block_max scratch, used before anything is staged
    stage2_tile<IW, Q>(a, xcd_tile(blockIdx.x, a.ngroups * a.n_ichunks * a.n_ttiles), lds, red, threadIdx.x);
}

template <int IW, int Q>
__global__ __launch_bounds__(kThreads) TX_S2_WAVES(IW, Q) void stage2_batch_kernel(const Stage2Args* __restrict__ jobs,
                                                                const int* __restrict__ prefix_base,
                                                                const int* __restrict__ info, uint32_t* queue) {
    extern __shared__ __align__(16) uint8_t lds[];
    int* red = reinterpret_cast<int*>(lds);
    const int njobs = info[0];
    if (njobs <= 0) return;
    const Stage2Args* cj = jobs + info[1];
    const int* prefix = prefix_base + info[2];
    for_each_claimed(prefix[njobs], queue, [&](int t) {
        const int jb = find_job(prefix, njobs, t);
        const Stage2Args a = cj[jb];
        int tv = static_cast<int>(threadIdx.x);
        asm volatile("" : "+v"(tv));
        stage2_tile<IW, Q>(a, t - prefix[jb], lds, red, tv);
    });
}

// ---------------------------------------------------------------------------
// Variants, geometry and launches.
// ---------------------------------------------------------------------------
static const Stage1Variant kS1[] = {{5, 4}, {7, 4}, {9, 4}, {5, 2}, {7, 2}, {9, 2}, {11, 2}, {13, 1}, {3, 4}};
static const Stage2Variant kS2[] = {{1}, {3}, {5}};
constexpr int kNS1 = sizeof(kS1) / sizeof(kS1[0]);
constexpr int kNS2 = sizeof(kS2) / sizeof(kS2[0]);
constexpr int kDefaultLds = 27296;        // first stage: a sixth of a CU's LDS (94 VGPRs hold it to 5 per CU)
constexpr int kDefaultLds2 = 32 * 1024;   // second stage
// Defaults: the fastest pair on the 4096-channel paper-scale block (first
// stage 9 output dwords per lane x 4 trials per wavefront at 27296 bytes, second
// stage 3 output dwords per lane at 32 KB); tx_plan_autotune measures per
// plan.  Q is odd in both stages (bank-conflict-free lane stride).
constexpr int kDefaultS1 = 2;
constexpr int kDefaultS2 = 1;

int stage1_variant_count() { return kNS1; }
int stage2_variant_count() { return kNS2; }
Stage1Variant stage1_variant(int v) { return kS1[v]; }
Stage2Variant stage2_variant(int v) { return kS2[v]; }

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
int device_max_lds();

// Trials per second-stage workgroup.  A workgroup computes all IW trials
// (padding repeats the last) and stages its sub-band rows once, which costs
// about as much as two trials: minimise chunks * (IW + 2).
static int pick_iw(int32_t g) {
    static const int cands[] = {16, 13, 8, 4, 2, 1};
    int best = 1;
    int64_t best_cost = INT64_MAX;
    for (int iw : cands) {
        const int64_t cost = (g + iw - 1) / iw * static_cast<int64_t>(iw + 2);
        if (cost < best_cost) {
            best_cost = cost;
            best = iw;
        }
    }
    return best;
}

DedispGeom dedisp_geometry(const tx_plan_s* p, int64_t nt, const Tiles& want) {
    DedispGeom g{};
    g.tiles = want;
    if (g.tiles.s1 < 0 || g.tiles.s1 >= kNS1) g.tiles.s1 = kDefaultS1;
    if (g.tiles.s2 < 0 || g.tiles.s2 >= kNS2) g.tiles.s2 = kDefaultS2;
    const Stage1Variant v1 = kS1[g.tiles.s1];
    const Stage2Variant v2 = kS2[g.tiles.s2];
    g.tt1 = 256 * v1.q;
    g.J1 = 4 * v1.jw;
    g.tt2 = 512 * v2.q;
    g.iw = pick_iw(p->g);
    const int iwp = (g.iw + 3) & ~3;

    // LDS: at least one row (and its table) per workgroup; stage 1 double
    // buffers when two fit in its LDS size.
    const int sp1 = plan_spread1(p, g.J1) + 15;
    const int W1 = ((sp1 >> 2) + 64 * v1.q + 1 + 3) & ~3;
    const int tabs1 = (p->m * (g.J1 + 1) * 4 + 15) & ~15;                            // shift tables
    const int need1 = std::max(4 * W1 + tabs1 + 48, kWaves * 512 * v1.q);   // a row and the tables; output pass
    g.lds1 = std::max(g.tiles.s1_lds > 0 ? g.tiles.s1_lds : kDefaultLds, need1);
    const int sp2 = plan_spread2(p, g.iw) + 7;
    const int W2 = ((sp2 >> 1) + 256 * v2.q + 1 + 3) & ~3;
    const int tabs2 = ((p->nsub + 3) & ~3) * iwp * 4;                                // shift table
    const int need2 = std::max(4 * (2 * W2 + 4) + tabs2 + 48, kWaves * 512 * v2.q);   // both copies of a row; output pass
    g.lds2 = std::max(g.tiles.s2_lds > 0 ? g.tiles.s2_lds : kDefaultLds2, need2);
    const int max_lds = device_max_lds();
    g.lds1 = std::min(g.lds1, std::max(need1, max_lds));
    g.lds2 = std::min(g.lds2, std::max(need2, max_lds));
    g.ok = g.lds1 <= max_lds && g.lds2 <= max_lds;
    g.tiles.s1_lds = g.lds1;
    g.tiles.s2_lds = g.lds2;

    g.n_ttiles2 = static_cast<int32_t>((nt + g.tt2 - 1) / g.tt2);
    // Stage 2 stages elements [start, start + 2 W + 8) of a series (copy 0
    // holds one 16-byte piece more than the W dwords the trials read), start
    // <= last tile start + max extent.
    const int64_t need = static_cast<int64_t>(std::max(g.n_ttiles2 - 1, 0)) * g.tt2 + p->max_extent + 2 * W2 + 8;
    g.B_pitch = round_up(std::max<int64_t>(need, nt + p->max_extent), g.tt1);
    g.n_ttiles1 = static_cast<int32_t>(g.B_pitch / g.tt1);
    g.n_jchunks = (p->ngroups + g.J1 - 1) / g.J1;
    g.n_ichunks = (p->g + g.iw - 1) / g.iw;
    g.ws_bytes = round_up(static_cast<int64_t>(p->ngroups) * p->nsub * g.B_pitch * 2, 256);
    return g;
}

// Raise a kernel's dynamic-LDS limit once, when a launch asks for more than
// the runtime's default; a failure leaves the limit (and the launch then fails
// with a reported error).
static void allow_lds(const void* fn, int bytes) {
    static std::mutex mu;
    static std::vector<std::pair<const void*, int>> done;
    if (bytes <= 64 * 1024) return;
    std::lock_guard<std::mutex> lock(mu);
    for (auto& d : done)
        if (d.first == fn && d.second >= bytes) return;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess)
        done.emplace_back(fn, bytes);
    (void)hipGetLastError();
}

int device_max_lds() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            cached = std::min(v, kMaxLds);
        else
            cached = 64 * 1024;
        (void)hipGetLastError();
    }
    return cached;
}

// Kernel tables: the single-job and the batch kernel of every variant.
struct KernelPair {
    const void* single;
    const void* batch;
};
#define TX_S1(Q, JW) {reinterpret_cast<const void*>(&stage1_kernel<Q, JW>), reinterpret_cast<const void*>(&stage1_batch_kernel<Q, JW>)}
static const KernelPair kS1Fn[kNS1] = {TX_S1(5, 4), TX_S1(7, 4), TX_S1(9, 4), TX_S1(5, 2), TX_S1(7, 2),
                                        TX_S1(9, 2), TX_S1(11, 2), TX_S1(13, 1), TX_S1(3, 4)};
#undef TX_S1
static const int kIW[] = {16, 13, 8, 4, 2, 1};
constexpr int kNIW = 6;
#define TX_S2(IW, Q) {reinterpret_cast<const void*>(&stage2_kernel<IW, Q>), reinterpret_cast<const void*>(&stage2_batch_kernel<IW, Q>)}
#define TX_S2Q(IW) TX_S2(IW, 1), TX_S2(IW, 3), TX_S2(IW, 5)
static const KernelPair kS2Fn[kNIW * kNS2] = {TX_S2Q(16), TX_S2Q(13), TX_S2Q(8), TX_S2Q(4), TX_S2Q(2), TX_S2Q(1)};
#undef TX_S2Q
#undef TX_S2

static const KernelPair* s2_pair(int iw, int variant) {
    for (int k = 0; k < kNIW; ++k)
        if (kIW[k] == iw) return &kS2Fn[k * kNS2 + variant];
    return nullptr;
}

static hipError_t launch(const void* fn, int grid, int lds, void** args, hipStream_t st) {
    allow_lds(fn, lds);
    const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, static_cast<size_t>(lds), st);
    return e != hipSuccess ? e : hipGetLastError();
}

void fill_stage_args(const tx_plan_s* p, const DedispGeom& geo, const uint8_t* d_in, int64_t in_pitch, int64_t nt,
                     int32_t* d_out, int64_t out_pitch, uint16_t* d_B, Stage1Args* s1, Stage2Args* s2) {
    *s1 = Stage1Args{};
    s1->x = d_in;
    s1->x_pitch = in_pitch;
    s1->x_len = nt + p->overlap;
    s1->x_off = 0;
    s1->mask = p->d_mask;
    s1->B = d_B;
    s1->B_pitch = geo.B_pitch;
    s1->dT = p->d_dT;
    s1->gpad = p->gpad;
    s1->nchan = p->nchan;
    s1->nsub = p->nsub;
    s1->m = p->m;
    s1->ngroups = p->ngroups;
    s1->n_jchunks = geo.n_jchunks;
    s1->n_ttiles = geo.n_ttiles1;
    s1->lds_bytes = geo.lds1;
    *s2 = Stage2Args{};
    s2->B = d_B;
    s2->B_pitch = geo.B_pitch;
    s2->Y = d_out;
    s2->y_pitch = out_pitch;
    s2->nt = nt;
    s2->rT = p->d_rT;
    s2->dpad = p->dpad;
    s2->ndm = p->ndm;
    s2->nsub = p->nsub;
    s2->g = p->g;
    s2->ngroups = p->ngroups;
    s2->n_ichunks = geo.n_ichunks;
    s2->n_ttiles = geo.n_ttiles2;
    s2->lds_bytes = geo.lds2;
    s2->flush = std::max(1, 65535 / (255 * p->m));
}

int64_t stage1_tiles(const Stage1Args& a) { return static_cast<int64_t>(a.nsub) * a.n_ttiles * a.n_jchunks; }
int64_t stage2_tiles(const Stage2Args& a) { return static_cast<int64_t>(a.ngroups) * a.n_ichunks * a.n_ttiles; }

hipError_t launch_dedisperse(const tx_plan_s* p, const DedispGeom& geo, const uint8_t* d_in, int64_t in_pitch,
                             int64_t nt, int32_t* d_out, int64_t out_pitch, uint16_t* d_B, hipStream_t stream,
                             int x_off) {
    if (!geo.ok || x_off < 0 || x_off > 15) return hipErrorInvalidValue;
    Stage1Args s1;
    Stage2Args s2;
    fill_stage_args(p, geo, d_in, in_pitch, nt, d_out, out_pitch, d_B, &s1, &s2);
    s1.x_off = x_off;
    void* a1[] = {&s1};
    int prof = prof_begin(TX_KERNEL_STAGE1, stream);
    hipError_t e = launch(kS1Fn[geo.tiles.s1].single, static_cast<int>(stage1_tiles(s1)), s1.lds_bytes, a1, stream);
    prof_end(prof, stream);
    if (e != hipSuccess) return e;
    const KernelPair* k2 = s2_pair(geo.iw, geo.tiles.s2);
    if (!k2) return hipErrorInvalidValue;
    void* a2[] = {&s2};
    prof = prof_begin(TX_KERNEL_STAGE2, stream);
    e = launch(k2->single, static_cast<int>(stage2_tiles(s2)), s2.lds_bytes, a2, stream);
    prof_end(prof, stream);
    return e;
}

// Workgroups of a kernel the device holds at once with `lds` bytes of dynamic
// LDS (0 if unknown), cached per (kernel, LDS size).
int resident_grid(const void* fn, int lds) {
    static std::mutex mu;
    static std::vector<std::pair<std::pair<const void*, int>, int>> done;
    std::lock_guard<std::mutex> lock(mu);
    for (auto& d : done)
        if (d.first.first == fn && d.first.second == lds) return d.second;
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kThreads, lds) != hipSuccess || cus <= 0 || per <= 0) {
        (void)hipGetLastError();
        return 0;
    }
    done.push_back({{fn, lds}, cus * per});
    return cus * per;
}

// A persistent batch launch: as many workgroups as the device holds at once,
// or `tiles` if fewer (0 = a graph that may later see any number of tiles).
static hipError_t launch_persistent(const void* fn, int lds, void** args, int64_t tiles, hipStream_t stream) {
    allow_lds(fn, lds);
    int grid = resident_grid(fn, lds);
    if (grid <= 0) grid = 256 * 4;
    if (tiles > 0 && tiles < grid) grid = static_cast<int>(tiles);
    const hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, static_cast<size_t>(lds), stream);
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_stage1_batch(int variant, int lds, const BatchRefs& r, int64_t tiles, hipStream_t stream) {
    if (variant < 0 || variant >= kNS1) return hipErrorInvalidValue;
    const void* fn = kS1Fn[variant].batch;
    const Stage1Args* jobs = static_cast<const Stage1Args*>(r.jobs);
    void* a[] = {&jobs, const_cast<const int**>(&r.prefix), const_cast<const int**>(&r.info),
                 const_cast<uint32_t**>(&r.queue)};
    const int prof = prof_begin(TX_KERNEL_STAGE1, stream);
    const hipError_t e = launch_persistent(fn, lds, a, tiles, stream);
    prof_end(prof, stream);
    return e;
}

hipError_t launch_stage2_batch(int iw, int variant, int lds, const BatchRefs& r, int64_t tiles, hipStream_t stream) {
    const KernelPair* k = (variant >= 0 && variant < kNS2) ? s2_pair(iw, variant) : nullptr;
    if (!k) return hipErrorInvalidValue;
    const Stage2Args* jobs = static_cast<const Stage2Args*>(r.jobs);
    void* a[] = {&jobs, const_cast<const int**>(&r.prefix), const_cast<const int**>(&r.info),
                 const_cast<uint32_t**>(&r.queue)};
    const int prof = prof_begin(TX_KERNEL_STAGE2, stream);
    const hipError_t e = launch_persistent(k->batch, lds, a, tiles, stream);
    prof_end(prof, stream);
    return e;
}

int stage2_iw(int32_t g) { return pick_iw(g); }

// ---------------------------------------------------------------------------
// Dedispersion without allocation.  The first-stage series of one chunk of
// output samples live in `scratch`, a file-scope device array that every GPU
// the library runs on holds until the process ends; the block is dedispersed
// chunk after chunk on the caller's stream (each chunk's two stages finish
// reading the array before the next chunk's first stage writes it, by stream
// order).  Every chunk reads its own window of the caller's rows (a 16-byte
// aligned base and a byte offset of 0..15) and writes its own output columns,
// so the result equals one tx_dedisperse of the whole block.  Calls that
// overlap on one GPU (other streams, other threads) share the array and race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[TX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// Device address of `scratch` on device `dev` (current): looked up once per
// device with hipGetSymbolAddress, since in host code the array's name is a
// host-side stand-in, not the device's copy.
static hipError_t noalloc_scratch(int dev, void** ptr) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

// Largest chunk (a multiple of the second-stage tile, at most nt) whose
// first-stage series fit `bytes` with tiles `t`, or 0 if not even one tile's
// do.  The scratch a chunk needs grows with its length.
static int64_t largest_chunk(const tx_plan_s* p, int64_t nt, const Tiles& t, int64_t bytes) {
    const DedispGeom g1 = dedisp_geometry(p, 1, t);
    if (!g1.ok || g1.ws_bytes > bytes) return 0;
    const int64_t tt2 = g1.tt2;
    int64_t lo = 1, hi = (nt + tt2 - 1) / tt2;       // whole tiles: lo fits
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (dedisp_geometry(p, std::min(nt, mid * tt2), t).ws_bytes <= bytes) lo = mid; else hi = mid - 1;
    }
    return std::min(nt, lo * tt2);
}

hipError_t launch_dedisperse_noalloc(const tx_plan_s* p, const Tiles& want, const uint8_t* d_in, int64_t in_pitch,
                                     int64_t nt, int32_t* d_out, int64_t out_pitch, hipStream_t stream, int dev,
                                     int64_t* need_bytes) {
    *need_bytes = 0;
    const int64_t cap = TX_NOALLOC_SCRATCH_BYTES;
    // The plan's tiles, else the first-stage variant (second stage kept) that
    // gives the longest chunk: a shorter first-stage tile shortens the series.
    Tiles best = want;
    int64_t chunk = largest_chunk(p, nt, want, cap);
    if (chunk < nt) {
        for (int v = 0; v < kNS1; ++v) {
            Tiles t = want;
            t.s1 = v;
            t.s1_lds = 0;
            const int64_t c = largest_chunk(p, nt, t, cap);
            if (c > chunk) {
                chunk = c;
                best = t;
            }
        }
    }
    if (chunk <= 0) {
        int64_t smallest = INT64_MAX;
        for (int v = 0; v < kNS1; ++v) {
            Tiles t = want;
            t.s1 = v;
            t.s1_lds = 0;
            const DedispGeom g = dedisp_geometry(p, 1, t);
            if (g.ok) smallest = std::min(smallest, g.ws_bytes);
        }
        *need_bytes = smallest == INT64_MAX ? -1 : smallest;
        return hipErrorInvalidValue;
    }
    void* ws = nullptr;
    hipError_t e = noalloc_scratch(dev, &ws);
    if (e != hipSuccess) return e;
    for (int64_t c0 = 0; c0 < nt; c0 += chunk) {
        const int64_t n = std::min(chunk, nt - c0);
        const DedispGeom geo = dedisp_geometry(p, n, best);
        if (!geo.ok || geo.ws_bytes > cap) return hipErrorInvalidValue;
        e = launch_dedisperse(p, geo, d_in + (c0 & ~int64_t(15)), in_pitch, n, d_out + c0, out_pitch,
                              static_cast<uint16_t*>(ws), stream, static_cast<int>(c0 & 15));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tx
