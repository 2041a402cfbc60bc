// Time downsampling of uint8 channel rows for gfx950, the step before each
// coarser-sampled DM range of a dedispersion plan (Sec. 2.3: downsampling
// before dedispersion in multiple DM ranges).
//
// out[c][t] = (sum of in[c][k t + i], i < k, + k / 2) / k  (integer division),
// the mean of k consecutive samples rounded to nearest, halves up, for k a
// power of two up to 64.  Pure data movement plus k - 1 adds per output:
// bound by HBM (k + 1 bytes per output).  A lane makes 16 outputs of one row
// from 16 k consecutive input bytes read as 16-byte loads, and writes them as
// one 16-byte store; the lanes of a wavefront walk one row.
#include "tx_internal.h"

namespace tx {

namespace {

// Sum of the 4 bytes of w (v_sad_u8 against zero).
__device__ __forceinline__ uint32_t byte_sum(uint32_t w) { return __builtin_amdgcn_sad_u8(w, 0u, 0u); }

template <int LOGK>
__global__ __launch_bounds__(256) void downsample_kernel(const uint8_t* __restrict__ in, int64_t in_pitch,
                                                         int32_t nchan, int64_t nt_out, uint8_t* __restrict__ out,
                                                         int64_t out_pitch, int64_t groups_per_row) {
    constexpr int K = 1 << LOGK;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t c = gid / groups_per_row;
    const int64_t g = gid - c * groups_per_row;
    if (c >= nchan) return;
    const int64_t t0 = 16 * g;                         // first output of this lane
    const int64_t n = min<int64_t>(16, nt_out - t0);   // outputs (1..16)
    const uint8_t* src = in + c * in_pitch + K * t0;
    uint32_t sums[16];
    if (n == 16) {
        if constexpr (K == 1) {
            const uint4 v = *reinterpret_cast<const uint4*>(src);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 16; ++j) sums[j] = (w[j >> 2] >> (8 * (j & 3))) & 255u;
        } else if constexpr (K == 2) {
            // Two 16-byte loads; pairs of bytes summed as 16-bit lanes.
            const uint4 a = *reinterpret_cast<const uint4*>(src);
            const uint4 b = *reinterpret_cast<const uint4*>(src + 16);
            const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const uint32_t p = (w[d] & 0x00FF00FFu) + ((w[d] >> 8) & 0x00FF00FFu);
                sums[2 * d] = p & 0xFFFFu;
                sums[2 * d + 1] = p >> 16;
            }
        } else {
            // K / 4 dwords per output; the lane's 16 K input bytes are K 16-byte loads.
            constexpr int DW = K / 4;
#pragma unroll
            for (int j = 0; j < 16; ++j) sums[j] = 0u;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const uint4 v = *reinterpret_cast<const uint4*>(src + 16 * q);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int dw = 4 * q + d;             // dword index within the lane's input
                    sums[dw / DW] += byte_sum(w[d]);
                }
            }
        }
    } else {
        // Row tail: bytes one by one (only the last lane of a row).
        for (int j = 0; j < 16; ++j) {
            uint32_t s = 0;
            if (j < n)
                for (int i = 0; i < K; ++i) s += src[K * j + i];
            sums[j] = s;
        }
    }
    uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < 16; ++j) o[j >> 2] |= ((sums[j] + K / 2) >> LOGK) << (8 * (j & 3));
    uint8_t* dst = out + c * out_pitch + t0;
    if (n == 16) {
        *reinterpret_cast<uint4*>(dst) = make_uint4(o[0], o[1], o[2], o[3]);
    } else {
        for (int j = 0; j < n; ++j) dst[j] = static_cast<uint8_t>(o[j >> 2] >> (8 * (j & 3)));
    }
}

template <int LOGK>
const void* downsample_fn() {
    return reinterpret_cast<const void*>(&downsample_kernel<LOGK>);
}

}  // namespace

hipError_t launch_downsample(const uint8_t* d_in, int64_t in_pitch, int32_t nchan, int64_t nt_out, int32_t k,
                             uint8_t* d_out, int64_t out_pitch, hipStream_t stream) {
    if (nchan < 1 || nt_out < 1) return hipSuccess;
    int logk = -1;
    for (int l = 0; l <= 6; ++l)
        if (k == (1 << l)) logk = l;
    if (logk < 0) return hipErrorInvalidValue;
    int64_t groups = (nt_out + 15) / 16;
    const int64_t blocks = (groups * nchan + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    static const void* const fns[7] = {downsample_fn<0>(), downsample_fn<1>(), downsample_fn<2>(), downsample_fn<3>(),
                                       downsample_fn<4>(), downsample_fn<5>(), downsample_fn<6>()};
    void* args[] = {&d_in, &in_pitch, &nchan, &nt_out, &d_out, &out_pitch, &groups};
    const int prof = prof_begin(TX_KERNEL_DOWNSAMPLE, stream);
    hipError_t e = hipLaunchKernel(fns[logk], dim3(static_cast<unsigned>(blocks)), dim3(256), args, 0, stream);
    prof_end(prof, stream);
    return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace tx
