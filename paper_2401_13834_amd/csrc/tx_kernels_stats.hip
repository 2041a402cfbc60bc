// Per-channel power sums of uint8 channel rows for gfx950, the statistics the
// paper's narrow-band RFI filter works on (Sec. 2.2: channels that are
// outliers in skewness and kurtosis across the band are removed).
//
// sums[c] = (sum x, sum x^2, sum x^3, sum x^4) over x = in[c][0 .. nt), exact
// in uint64.  A workgroup reduces one chunk of one row: lanes read 16-byte
// pieces (coalesced along the row), sum 4 bytes at a time with v_sad_u8 and
// v_dot4_u32_u8 (sum of squares), and the cubes and fourth powers byte by
// byte; the workgroup's totals go to the row with 64-bit atomic adds.  Bound:
// HBM for reads, with about 3 VALU operations per byte.
#include "tx_internal.h"

namespace tx {

namespace {

constexpr int kChunk = 16384;   // samples per workgroup

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(256) void power_sums_kernel(const uint8_t* __restrict__ in, int64_t in_pitch,
                                                         int64_t nt, int32_t nchunks,
                                                         unsigned long long* __restrict__ sums) {
    __shared__ unsigned long long red[4][4];
    const int c = blockIdx.x / nchunks;
    const int k = blockIdx.x - c * nchunks;
    const int64_t t0 = static_cast<int64_t>(k) * kChunk;
    const int64_t t1 = min<int64_t>(nt, t0 + kChunk);
    const uint8_t* row = in + static_cast<int64_t>(c) * in_pitch;
    unsigned long long s1 = 0, s2 = 0, s3 = 0, s4 = 0;
    for (int64_t t = t0 + 16 * static_cast<int64_t>(threadIdx.x); t < t1; t += 16 * 256) {
        uint32_t w[4];
        if (t + 16 <= t1) {
            const uint4 v = *reinterpret_cast<const uint4*>(row + t);
            w[0] = v.x;
            w[1] = v.y;
            w[2] = v.z;
            w[3] = v.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) w[j] = 0u;
            for (int j = 0; t + j < t1; ++j) w[j >> 2] |= static_cast<uint32_t>(row[t + j]) << (8 * (j & 3));
        }
        uint32_t a1 = 0, a2 = 0, a3 = 0;   // per 16 bytes: < 2^12, 2^20, 2^28
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a1 = __builtin_amdgcn_sad_u8(w[j], 0u, a1);
            a2 = __builtin_amdgcn_udot4(w[j], w[j], a2, false);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t x = (w[j] >> (8 * b)) & 255u;
                const uint32_t x2 = x * x;
                a3 += x2 * x;
                s4 += static_cast<unsigned long long>(x2) * x2;
            }
        }
        s1 += a1;
        s2 += a2;
        s3 += a3;
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    s3 = wave_sum(s3);
    s4 = wave_sum(s4);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[wave][0] = s1;
        red[wave][1] = s2;
        red[wave][2] = s3;
        red[wave][3] = s4;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const unsigned long long v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                                     red[3][threadIdx.x];
        atomicAdd(&sums[4 * c + threadIdx.x], v);
    }
}

__global__ void zero_sums_kernel(unsigned long long* __restrict__ sums, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) sums[i] = 0ull;
}

}  // namespace

hipError_t launch_power_sums(const uint8_t* d_in, int64_t in_pitch, int32_t nchan, int64_t nt, uint64_t* d_sums,
                             hipStream_t stream) {
    if (nchan < 1) return hipSuccess;
    unsigned long long* sums = reinterpret_cast<unsigned long long*>(d_sums);
    const int64_t n4 = 4 * static_cast<int64_t>(nchan);
    hipLaunchKernelGGL(zero_sums_kernel, dim3(static_cast<unsigned>((n4 + 255) / 256)), dim3(256), 0, stream, sums, n4);
    if (nt > 0) {
        const int64_t nchunks = (nt + kChunk - 1) / kChunk;
        const int64_t grid = nchunks * nchan;
        if (grid > INT32_MAX) return hipErrorInvalidValue;
        hipLaunchKernelGGL(power_sums_kernel, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, d_in, in_pitch,
                           nt, static_cast<int32_t>(nchunks), sums);
    }
    return hipGetLastError();
}

}  // namespace tx
