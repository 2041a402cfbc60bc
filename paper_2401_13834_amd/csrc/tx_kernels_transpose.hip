// Time-major to channel-major transpose of uint8 filterbank samples for
// gfx950: the "transpose" step of the paper's dedispersion data flow (Sec. 2.3,
// Fig. "dedispersion_flow"), which turns blocks as recorded (one row of
// channels per time sample) into the channel rows the first stage reads.
//
// Pure data movement, so the bound is HBM: every byte is read once and
// written once.  A workgroup moves a 128-channel x 128-sample tile:
// * loads: lane (c16, t4) reads 16 channels of 4 consecutive time rows as
//   16-byte loads; 8 lanes cover one 128-byte line of a time row;
// * a 4 x 4 byte transpose in registers (v_perm) turns each 4 x 4 block into 4
//   dwords of 4 time samples of one channel;
// * the dwords go to an LDS tile [channel][time] whose 16-byte groups are
//   XOR-swizzled by channel, so that the 4-byte writes of lanes with different
//   channel groups land in different banks while each row's 16-byte groups
//   stay aligned for 16-byte reads;
// * stores: 8 lanes write one 128-byte run of a channel row as 16-byte stores.
#include "tx_internal.h"

namespace tx {

namespace {

constexpr int kTC = 128;   // channels per tile
constexpr int kTT = 128;   // time samples per tile
constexpr int kRowDw = kTT / 4;

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// Bytes k of the 4 words r0..r3 (time rows) as one word, time in byte order.
__device__ __forceinline__ void transpose4x4(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3, uint32_t o[4]) {
    // Pairs first: (r0, r1) interleaved by bytes, then by 16-bit halves.
    const uint32_t a = perm(r1, r0, 0x05010400u);   // r0.b0 r1.b0 r0.b1 r1.b1
    const uint32_t b = perm(r1, r0, 0x07030602u);   // r0.b2 r1.b2 r0.b3 r1.b3
    const uint32_t c = perm(r3, r2, 0x05010400u);
    const uint32_t d = perm(r3, r2, 0x07030602u);
    o[0] = perm(c, a, 0x05040100u);                 // r0.b0 r1.b0 r2.b0 r3.b0
    o[1] = perm(c, a, 0x07060302u);                 // byte 1 of every row
    o[2] = perm(d, b, 0x05040100u);
    o[3] = perm(d, b, 0x07060302u);
}

// Physical dword column of logical column `col` in tile row `row`: the 16-byte
// group index is XORed with bits 4..6 of the row (the lane's channel group).
__device__ __forceinline__ int swz(int row, int col) { return col ^ (((row >> 4) & 7) << 2); }

__device__ __forceinline__ int xcd_tile_t(int bid, int total) {
    const int nx = 8;
    const int x = bid % nx, k = bid / nx;
    const int q = total / nx, r = total % nx;
    return x * q + min(x, r) + k;
}

__global__ __launch_bounds__(256) void transpose_tf_kernel(const uint8_t* __restrict__ in, int64_t in_pitch,
                                                           int32_t nchan, int64_t nt, uint8_t* __restrict__ out,
                                                           int64_t out_pitch, int32_t n_ctiles, int32_t n_tiles) {
    __shared__ __align__(16) uint32_t tile[kTC * kRowDw];
    const int t = xcd_tile_t(blockIdx.x, n_tiles);
    const int ct = t % n_ctiles;
    const int tt = t / n_ctiles;
    const int c0 = ct * kTC;
    const int64_t t0 = static_cast<int64_t>(tt) * kTT;
    const int tid = threadIdx.x;

    // Load 4 time rows x 16 channels per lane.
    {
        const int c16 = tid & 7, t4 = tid >> 3;   // 8 channel groups x 32 row quads
        const int cb = c0 + 16 * c16;
        uint32_t w[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t ti = t0 + 4 * t4 + r;
            const uint8_t* src = in + ti * in_pitch + cb;
            if (ti < nt && cb + 16 <= nchan) {
                const uint4 v = *reinterpret_cast<const uint4*>(src);
                w[r][0] = v.x;
                w[r][1] = v.y;
                w[r][2] = v.z;
                w[r][3] = v.w;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) w[r][k] = 0u;
                if (ti < nt)
                    for (int k = 0; k < 16; ++k)
                        if (cb + k < nchan) w[r][k >> 2] |= static_cast<uint32_t>(src[k]) << (8 * (k & 3));
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t o[4];
            transpose4x4(w[0][j], w[1][j], w[2][j], w[3][j], o);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int row = 16 * c16 + 4 * j + k;
                tile[row * kRowDw + swz(row, t4)] = o[k];
            }
        }
    }
    __syncthreads();

    // Store: lane (g, row) writes 16 time samples of one channel.
#pragma unroll
    for (int pass = 0; pass < kTC * (kTT / 16) / 256; ++pass) {
        const int idx = pass * 256 + tid;
        const int g = idx & 7, row = idx >> 3;
        const int c = c0 + row;
        const int64_t ts = t0 + 16 * g;
        if (c >= nchan || ts >= nt) continue;
        const uint4 v = *reinterpret_cast<const uint4*>(&tile[row * kRowDw + swz(row, 4 * g)]);
        uint8_t* dst = out + static_cast<int64_t>(c) * out_pitch + ts;
        if (ts + 16 <= nt) {
            *reinterpret_cast<uint4*>(dst) = v;
        } else {
            const uint32_t d[4] = {v.x, v.y, v.z, v.w};
            for (int k = 0; k < 16 && ts + k < nt; ++k) dst[k] = static_cast<uint8_t>(d[k >> 2] >> (8 * (k & 3)));
        }
    }
}

}  // namespace

hipError_t launch_transpose_tf(const uint8_t* d_tf, int64_t tf_pitch, int32_t nchan, int64_t nt, uint8_t* d_ft,
                               int64_t ft_pitch, hipStream_t stream) {
    if (nchan < 1 || nt < 1) return hipSuccess;
    const int64_t n_ct = (nchan + kTC - 1) / kTC;
    const int64_t n_tt = (nt + kTT - 1) / kTT;
    const int64_t total = n_ct * n_tt;
    if (total > INT32_MAX) return hipErrorInvalidValue;
    const int prof = prof_begin(TX_KERNEL_TRANSPOSE, stream);
    hipLaunchKernelGGL(transpose_tf_kernel, dim3(static_cast<unsigned>(total)), dim3(256), 0, stream, d_tf, tf_pitch,
                       nchan, nt, d_ft, ft_pitch, static_cast<int32_t>(n_ct), static_cast<int32_t>(total));
    prof_end(prof, stream);
    return hipGetLastError();
}

}  // namespace tx
