// Measured peaks of the units the dedispersion kernels use, on the current
// GPU: HBM copy bandwidth (one and several 16-byte loads in flight per
// thread) and read-only bandwidth, 32-bit and packed 16-bit integer add rates, the
// issue rates of the three-operand add, byte-align and byte-permute
// instructions, and LDS read bandwidth and cost per read instruction
// (aligned 4-, 8- and 16-byte reads, the first stage's paired 4-byte reads,
// and 4-byte reads off dword alignment).  Prints one JSON object.
//
//   tx_peaks [--quick]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#define CHECK(x)                                                                              \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));               \
            std::exit(1);                                                                     \
        }                                                                                     \
    } while (0)

constexpr int kThreads = 256;
constexpr int kAcc = 16;

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(kThreads) void add32_kernel(const uint32_t* in, uint32_t* out, int iters) {
    uint32_t a[kAcc];
    const uint32_t x = in[threadIdx.x & 63], y = in[(threadIdx.x + 7) & 63];
#pragma unroll
    for (int k = 0; k < kAcc; ++k) a[k] = x + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kAcc; ++k) a[k] += a[(k + 1) % kAcc];
    }
    uint32_t r = y;
#pragma unroll
    for (int k = 0; k < kAcc; ++k) r ^= a[k];
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

__global__ __launch_bounds__(kThreads) void add16x2_kernel(const uint32_t* in, uint32_t* out, int iters) {
    u16x2 a[kAcc];
    u16x2 x, y;
    __builtin_memcpy(&x, &in[threadIdx.x & 63], 4);
    __builtin_memcpy(&y, &in[(threadIdx.x + 5) & 63], 4);
#pragma unroll
    for (int k = 0; k < kAcc; ++k) a[k] = x + (unsigned short)k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kAcc; ++k) a[k] += a[(k + 1) % kAcc];
    }
    uint32_t r = 0;
    __builtin_memcpy(&r, &y, 4);
#pragma unroll
    for (int k = 0; k < kAcc; ++k) {
        uint32_t v;
        __builtin_memcpy(&v, &a[k], 4);
        r ^= v;
    }
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

// One byte permute and one 32-bit add per step: the inner pattern of the
// first dedispersion stage.
__global__ __launch_bounds__(kThreads) void perm_add_kernel(const uint32_t* in, uint32_t* out, int iters) {
    uint32_t a[kAcc];
    const uint32_t x = in[threadIdx.x & 63], y = in[(threadIdx.x + 3) & 63];
    const uint32_t sel = 0x0C030C01u + (in[0] & 3u) * 0x00010001u;
#pragma unroll
    for (int k = 0; k < kAcc; ++k) a[k] = k ^ y;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kAcc; ++k) a[k] += __builtin_amdgcn_perm(a[(k + 1) % kAcc], a[k] ^ x, sel);
    }
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < kAcc; ++k) r ^= a[k];
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

// Issue rates of the three-operand (VOP3) instructions of the first stage's
// inner loop, one instruction per step, 16 independent chains per lane:
// v_add3_u32 (kind 0), v_alignbyte_b32 (kind 1), v_perm_b32 (kind 2).
template <int KIND>
__global__ __launch_bounds__(kThreads) void vop3_kernel(const uint32_t* in, uint32_t* out, int iters) {
    uint32_t a[kAcc];
    const uint32_t x = in[threadIdx.x & 63];
    const uint32_t sel = KIND == 1 ? (in[1] & 3u) : 0x0C030C01u + (in[0] & 3u) * 0x00010001u;
#pragma unroll
    for (int k = 0; k < kAcc; ++k) a[k] = x ^ (k * 0x01010101u);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kAcc; ++k) {
            if constexpr (KIND == 0) a[k] = a[k] + a[(k + 1) % kAcc] + x;
            else if constexpr (KIND == 1) a[k] = __builtin_amdgcn_alignbyte(a[(k + 1) % kAcc], a[k], sel);
            else a[k] = __builtin_amdgcn_perm(a[(k + 1) % kAcc], a[k], sel);
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < kAcc; ++k) r ^= a[k];
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

// LDS reads: every lane reads W consecutive bytes (W = 4, 8, 16) at a
// conflict-free address, `reps` times over a 16 KiB buffer.
template <int W>
__global__ __launch_bounds__(kThreads) void lds_kernel(uint32_t* out, int iters) {
    __shared__ __align__(16) uint32_t buf[4096];
    for (int i = threadIdx.x; i < 4096; i += kThreads) buf[i] = i * 2654435761u;
    __syncthreads();
    constexpr int D = W / 4;
    uint32_t acc = 0;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int base = (wave * 64 * D) & 4095;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = (base + lane * D + u * 256 * D) & (4096 - D);
            if constexpr (D == 1) {
                acc += buf[idx];
            } else if constexpr (D == 2) {
                const uint2 v = *reinterpret_cast<const uint2*>(&buf[idx]);
                acc += v.x ^ v.y;
            } else {
                const uint4 v = *reinterpret_cast<const uint4*>(&buf[idx]);
                acc += v.x ^ v.y ^ v.z ^ v.w;
            }
        }
        base = (base + 64) & 4095;
    }
    out[blockIdx.x * kThreads + threadIdx.x] = acc;
}

// LDS reads in the first stage's form: every lane reads 10 consecutive dwords
// (as five paired 4-byte reads) at a lane stride of 9 dwords, from a
// 16-dword aligned base; indices stay below 3072 + 63 * 9 + 10 < 4096 + 16.
__global__ __launch_bounds__(kThreads) void lds_stride9_kernel(uint32_t* out, int iters) {
    __shared__ __align__(16) uint32_t buf[4096 + 16];
    for (int i = threadIdx.x; i < 4096 + 16; i += kThreads) buf[i] = i * 2654435761u;
    __syncthreads();
    uint32_t acc = 0;
    const int lane = threadIdx.x & 63;
    int base = (threadIdx.x >> 6) * 256;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t* p = buf + ((base + u * 1024) & 3072) + 9 * lane + (i & 1);
#pragma unroll
            for (int c = 0; c < 10; ++c) acc += p[c];
        }
        base = (base + 64) & 4095;
    }
    out[blockIdx.x * kThreads + threadIdx.x] = acc;
}

// 4-byte LDS reads at a byte offset `off` (1..3) from a dword boundary,
// consecutive lanes at consecutive dwords.  The first pass counts reads that
// do not return the four bytes that follow the address.  The last byte read is
// below 4 * (3072 + 63 + 1) + 3 < 4 * 4160.
__device__ __forceinline__ uint32_t lds_pattern(int b) { return static_cast<uint32_t>((b * 37 + (b >> 8) * 11) & 0xFF); }

__global__ __launch_bounds__(kThreads) void lds_unaligned_kernel(uint32_t* out, uint32_t* wrong, int iters, int off) {
    __shared__ __align__(16) uint32_t buf[4160];
    uint8_t* b8 = reinterpret_cast<uint8_t*>(buf);
    for (int i = threadIdx.x; i < 4 * 4160; i += kThreads) b8[i] = static_cast<uint8_t>(lds_pattern(i));
    __syncthreads();
    uint32_t acc = 0, bad = 0;
    const int lane = threadIdx.x & 63;
    int base = (threadIdx.x >> 6) * 256;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int at = 4 * (((base + u * 1024) & 3072) + lane) + off;
            const uint32_t v = *reinterpret_cast<const uint32_t*>(b8 + at);
            acc += v;
            if (i == 0)
                bad += v != (lds_pattern(at) | lds_pattern(at + 1) << 8 | lds_pattern(at + 2) << 16 |
                             lds_pattern(at + 3) << 24);
        }
        base = (base + 64) & 4095;
    }
    out[blockIdx.x * kThreads + threadIdx.x] = acc;
    if (bad) atomicAdd(wrong, bad);
}

// Issue rates of single VALU forms: each instruction issued from inline asm
// (arithmetic only), 8 independent chains per lane, 32 per loop step.
// Kinds: 0 v_add_u32, 1 v_add3_u32, 2 v_alignbyte_b32, 3 v_perm_b32,
// 4 v_pk_add_u16, 5 v_add_u32 with SDWA byte/word selects, 6 v_add_f32,
// 7 v_fma_f32, 8 v_fma_mix_f32 (float16 operand), 9 v_add_f64, 10 v_max_f64.
constexpr int kIssueKinds = 11;
template <int KIND>
__global__ __launch_bounds__(kThreads) void issue_kernel(const uint32_t* in, uint32_t* out, int iters) {
    uint32_t a[8];
    double d[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = in[i];
        d[i] = static_cast<double>(in[i]);
    }
    const uint32_t b = in[16], c = in[17];
    const double db = static_cast<double>(in[18]);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if constexpr (KIND == 0) asm volatile("v_add_u32_e32 %0, %1, %0" : "+v"(a[i]) : "v"(b));
                else if constexpr (KIND == 1) asm volatile("v_add3_u32 %0, %1, %2, %0" : "+v"(a[i]) : "v"(b), "v"(c));
                else if constexpr (KIND == 2) asm volatile("v_alignbyte_b32 %0, %1, %0, %2" : "+v"(a[i]) : "v"(b), "v"(c));
                else if constexpr (KIND == 3) asm volatile("v_perm_b32 %0, %1, %0, %2" : "+v"(a[i]) : "v"(b), "v"(c));
                else if constexpr (KIND == 4) asm volatile("v_pk_add_u16 %0, %1, %0" : "+v"(a[i]) : "v"(b));
                else if constexpr (KIND == 5)
                    asm volatile("v_add_u32_sdwa %0, %1, %0 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:BYTE_2 "
                                 "src1_sel:WORD_1"
                                 : "+v"(a[i])
                                 : "v"(b));
                else if constexpr (KIND == 6) asm volatile("v_add_f32_e32 %0, %1, %0" : "+v"(a[i]) : "v"(b));
                else if constexpr (KIND == 7) asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(a[i]) : "v"(b), "v"(c));
                else if constexpr (KIND == 8)
                    asm volatile("v_fma_mix_f32 %0, %1, %2, %0 op_sel_hi:[1,0,0]" : "+v"(a[i]) : "v"(b), "v"(c));
                else if constexpr (KIND == 9) asm volatile("v_add_f64 %0, %1, %0" : "+v"(d[i]) : "v"(db));
                else asm volatile("v_max_f64 %0, %1, %0" : "+v"(d[i]) : "v"(db));
            }
    }
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) x ^= a[i] ^ static_cast<uint32_t>(__double_as_longlong(d[i]));
    out[blockIdx.x * kThreads + threadIdx.x] = x;
}

// LDS writes: every lane writes W bytes (W = 4, 8, 16) at natural alignment,
// consecutive lanes at consecutive addresses; indices below 3072 + 64 * 4.
template <int W>
__global__ __launch_bounds__(kThreads) void lds_write_kernel(uint32_t* out, int iters) {
    __shared__ __align__(16) uint32_t buf[4096 + 16];
    constexpr int D = W / 4;
    const int lane = threadIdx.x & 63;
    int base = (threadIdx.x >> 6) * 256;
    uint32_t x = threadIdx.x;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int idx = ((base + u * 1024) & 3072) + D * lane;
            if constexpr (D == 4) *reinterpret_cast<uint4*>(&buf[idx]) = make_uint4(x, x + 1, x + 2, x + 3);
            else if constexpr (D == 2) *reinterpret_cast<uint2*>(&buf[idx]) = make_uint2(x, x + 1);
            else buf[idx] = x;
            x += 5;
        }
        base = (base + 64) & 4095;
    }
    __syncthreads();
    out[blockIdx.x * kThreads + threadIdx.x] = buf[threadIdx.x * 4];
}

// 16-byte LDS reads 4 bytes past a 16-byte boundary (the form an arbitrary
// dword shift would need), lanes 16 bytes apart.  Indices stay below
// 3072 + 63 * 4 + 1 + 4 < 4096 + 16.
__global__ __launch_bounds__(kThreads) void lds_b128_off4_kernel(uint32_t* out, int iters) {
    __shared__ __align__(16) uint32_t buf[4096 + 16];
    for (int i = threadIdx.x; i < 4096 + 16; i += kThreads) buf[i] = i * 2654435761u;
    __syncthreads();
    uint32_t acc = 0;
    const int lane = threadIdx.x & 63;
    int base = (threadIdx.x >> 6) * 256;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int idx = ((base + u * 1024) & 3072) + 4 * lane + 1;
            const uint4 v = *static_cast<const uint4*>(__builtin_assume_aligned(&buf[idx], 16));
            acc += v.x ^ v.y ^ v.z ^ v.w;
        }
        base = (base + 64) & 4095;
    }
    out[blockIdx.x * kThreads + threadIdx.x] = acc;
}

__global__ void copy_kernel(const uint4* __restrict__ in, uint4* __restrict__ out, size_t n) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) out[i] = in[i];
}

// The same copy with U independent 16-byte loads in flight per thread before
// their stores (pieces i, i + stride, ..., i + (U - 1) stride), then the
// pieces left over one at a time.  More bytes in flight per CU than the plain
// copy, whose one outstanding load per thread can leave HBM waiting on latency.
template <int U>
__global__ void copy_u_kernel(const uint4* __restrict__ in, uint4* __restrict__ out, size_t n) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = in[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) out[i + u * stride] = v[u];
    }
    for (; i < n; i += stride) out[i] = in[i];
}

// Read-only stream: U independent 16-byte loads per thread per step, folded
// into one word per thread that is stored at the end (so no load is dropped).
template <int U>
__global__ void read_u_kernel(const uint4* __restrict__ in, size_t n, uint32_t* __restrict__ out) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = in[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n; i += stride) acc ^= in[i].x;
    out[blockIdx.x * (size_t)blockDim.x + threadIdx.x] = acc;
}

template <typename F>
static float time_ms(F f, int reps) {
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    f();
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(a));
    for (int r = 0; r < reps; ++r) f();
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, a, b));
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
    return ms / reps;
}

int main(int argc, char** argv) {
    const bool quick = argc > 1 && std::strcmp(argv[1], "--quick") == 0;
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    const double clk_hz = prop.clockRate * 1e3;
    const int blocks = cus * 8;
    uint32_t *in, *out;
    CHECK(hipMalloc(&in, 64 * 4));
    CHECK(hipMalloc(&out, (size_t)blocks * kThreads * 4));
    std::vector<uint32_t> h(64);
    for (int i = 0; i < 64; ++i) h[i] = 0x01020304u * (i + 1);
    CHECK(hipMemcpy(in, h.data(), 256, hipMemcpyHostToDevice));
    const int iters = quick ? 2000 : 20000;
    const double lanes = (double)blocks * kThreads;

    float t_add = time_ms([&] { hipLaunchKernelGGL(add32_kernel, dim3(blocks), dim3(kThreads), 0, 0, in, out, iters); }, 3);
    const double add32 = lanes * iters * kAcc / (t_add * 1e-3);
    float t_pk = time_ms([&] { hipLaunchKernelGGL(add16x2_kernel, dim3(blocks), dim3(kThreads), 0, 0, in, out, iters); }, 3);
    const double add16 = 2.0 * lanes * iters * kAcc / (t_pk * 1e-3);
    float t_perm = time_ms([&] { hipLaunchKernelGGL(perm_add_kernel, dim3(blocks), dim3(kThreads), 0, 0, in, out, iters); }, 3);
    const double perm_add = lanes * iters * kAcc / (t_perm * 1e-3);   // (perm + add) pairs per second

    float t_v3[3];
    t_v3[0] = time_ms([&] { hipLaunchKernelGGL(vop3_kernel<0>, dim3(blocks), dim3(kThreads), 0, 0, in, out, iters); }, 3);
    t_v3[1] = time_ms([&] { hipLaunchKernelGGL(vop3_kernel<1>, dim3(blocks), dim3(kThreads), 0, 0, in, out, iters); }, 3);
    t_v3[2] = time_ms([&] { hipLaunchKernelGGL(vop3_kernel<2>, dim3(blocks), dim3(kThreads), 0, 0, in, out, iters); }, 3);
    double v3_rate[3];
    for (int k = 0; k < 3; ++k) v3_rate[k] = lanes * iters * kAcc / (t_v3[k] * 1e-3) / cus / clk_hz;

    const int lit = quick ? 2000 : 20000;
    float t_l4 = time_ms([&] { hipLaunchKernelGGL(lds_kernel<4>, dim3(blocks), dim3(kThreads), 0, 0, out, lit); }, 3);
    float t_l8 = time_ms([&] { hipLaunchKernelGGL(lds_kernel<8>, dim3(blocks), dim3(kThreads), 0, 0, out, lit); }, 3);
    float t_l16 = time_ms([&] { hipLaunchKernelGGL(lds_kernel<16>, dim3(blocks), dim3(kThreads), 0, 0, out, lit); }, 3);
    auto lds_bw = [&](float ms, int w) { return lanes * lit * 8.0 * w / (ms * 1e-3); };
    // clocks per wave-level read instruction per CU (reads of one wavefront)
    auto lds_clk = [&](float ms, double wave_reads) { return ms * 1e-3 * clk_hz * cus / wave_reads; };
    const double waves = (double)blocks * kThreads / 64;
    float t_s9 = time_ms([&] { hipLaunchKernelGGL(lds_stride9_kernel, dim3(blocks), dim3(kThreads), 0, 0, out, lit); }, 3);
    uint32_t* wrong;
    CHECK(hipMalloc(&wrong, 4));
    CHECK(hipMemset(wrong, 0, 4));
    const int uit = lit / 8;
    float t_ua = time_ms([&] { hipLaunchKernelGGL(lds_unaligned_kernel, dim3(blocks), dim3(kThreads), 0, 0, out, wrong,
                                                  uit, 1); }, 3);
    uint32_t n_wrong = 0;
    CHECK(hipMemcpy(&n_wrong, wrong, 4, hipMemcpyDeviceToHost));
    CHECK(hipFree(wrong));

    float t_is[kIssueKinds];
    {
        std::vector<uint32_t> hv(64);
        for (int i = 0; i < 64; ++i) hv[i] = 0x3f800000u + 3u * i;   // small positive floats as bits
        CHECK(hipMemcpy(in, hv.data(), 256, hipMemcpyHostToDevice));
        const int it2 = quick ? 2000 : 20000;
        auto run_is = [&](auto kern) {
            return time_ms([&] { hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), 0, 0, in, out, it2); }, 3);
        };
        t_is[0] = run_is(issue_kernel<0>);
        t_is[1] = run_is(issue_kernel<1>);
        t_is[2] = run_is(issue_kernel<2>);
        t_is[3] = run_is(issue_kernel<3>);
        t_is[4] = run_is(issue_kernel<4>);
        t_is[5] = run_is(issue_kernel<5>);
        t_is[6] = run_is(issue_kernel<6>);
        t_is[7] = run_is(issue_kernel<7>);
        t_is[8] = run_is(issue_kernel<8>);
        t_is[9] = run_is(issue_kernel<9>);
        t_is[10] = run_is(issue_kernel<10>);
        for (int k = 0; k < kIssueKinds; ++k) t_is[k] = static_cast<float>(lanes * it2 * 32 / (t_is[k] * 1e-3) / cus / clk_hz);
    }
    float t_w4 = time_ms([&] { hipLaunchKernelGGL(lds_write_kernel<4>, dim3(blocks), dim3(kThreads), 0, 0, out, lit); }, 3);
    float t_w8 = time_ms([&] { hipLaunchKernelGGL(lds_write_kernel<8>, dim3(blocks), dim3(kThreads), 0, 0, out, lit); }, 3);
    float t_w16 = time_ms([&] { hipLaunchKernelGGL(lds_write_kernel<16>, dim3(blocks), dim3(kThreads), 0, 0, out, lit); }, 3);
    float t_r16o = time_ms([&] { hipLaunchKernelGGL(lds_b128_off4_kernel, dim3(blocks), dim3(kThreads), 0, 0, out, uit); }, 3);

    const size_t bytes = (size_t)(quick ? 1 : 4) << 30;
    uint4 *src, *dst;
    CHECK(hipMalloc(&src, bytes));
    CHECK(hipMalloc(&dst, bytes));
    CHECK(hipMemset(src, 1, bytes));
    const size_t n = bytes / 16;
    float t_cp = time_ms([&] { hipLaunchKernelGGL(copy_kernel, dim3(cus * 16), dim3(256), 0, 0, src, dst, n); }, 5);
    const double copy_bw = 2.0 * bytes / (t_cp * 1e-3);
    // Copies and read-only streams with 4 or 8 loads in flight per thread, on
    // grids of 8 and 32 workgroups of 256 threads per CU: the best of each.
    const int grids[2] = {cus * 8, cus * 32};
    uint32_t* sink;
    CHECK(hipMalloc(&sink, (size_t)grids[1] * 256 * sizeof(uint32_t)));
    double copy_u_bw = 0.0, read_u_bw = 0.0;
    int copy_u_best[2] = {0, 0}, read_u_best[2] = {0, 0};
    for (int gi = 0; gi < 2; ++gi) {
        const int gb = grids[gi];
        const float c4 = time_ms([&] { hipLaunchKernelGGL(copy_u_kernel<4>, dim3(gb), dim3(256), 0, 0, src, dst, n); }, 5);
        const float c8 = time_ms([&] { hipLaunchKernelGGL(copy_u_kernel<8>, dim3(gb), dim3(256), 0, 0, src, dst, n); }, 5);
        const float r4 = time_ms([&] { hipLaunchKernelGGL(read_u_kernel<4>, dim3(gb), dim3(256), 0, 0, src, n, sink); }, 5);
        const float r8 = time_ms([&] { hipLaunchKernelGGL(read_u_kernel<8>, dim3(gb), dim3(256), 0, 0, src, n, sink); }, 5);
        const float cs[2] = {c4, c8}, rs[2] = {r4, r8};
        for (int k = 0; k < 2; ++k) {
            const double cb = 2.0 * bytes / (cs[k] * 1e-3), rb = 1.0 * bytes / (rs[k] * 1e-3);
            if (cb > copy_u_bw) {
                copy_u_bw = cb;
                copy_u_best[0] = 4 << k;
                copy_u_best[1] = gb / cus;
            }
            if (rb > read_u_bw) {
                read_u_bw = rb;
                read_u_best[0] = 4 << k;
                read_u_best[1] = gb / cus;
            }
        }
    }
    CHECK(hipFree(sink));

    std::printf("{\"device\": \"%s\", \"cus\": %d, \"clock_mhz\": %.0f, "
                "\"add32_per_s\": %.4e, \"add16_packed_per_s\": %.4e, \"perm_add_pairs_per_s\": %.4e, "
                "\"add32_per_clk_per_cu\": %.2f, \"add16_per_clk_per_cu\": %.2f, "
                "\"lds_b32_bytes_per_s\": %.4e, \"lds_b64_bytes_per_s\": %.4e, \"lds_b128_bytes_per_s\": %.4e, "
                "\"lds_b128_bytes_per_clk_per_cu\": %.1f, \"lds_b32_bytes_per_clk_per_cu\": %.1f, "
                "\"add3_per_clk_per_cu\": %.2f, \"alignbyte_per_clk_per_cu\": %.2f, \"perm_per_clk_per_cu\": %.2f, "
                "\"lds_clk_per_wave_read\": {\"b32\": %.2f, \"b64\": %.2f, \"b128\": %.2f, "
                "\"paired_b32_stride9\": %.2f, \"b32_byte_offset1\": %.2f, \"b128_dword_offset1\": %.2f}, "
                "\"lds_b32_byte_offset1_wrong\": %u, "
                "\"lds_clk_per_wave_write\": {\"b32\": %.2f, \"b64\": %.2f, \"b128\": %.2f}, "
                "\"issue_lane_instr_per_clk_per_cu\": {\"v_add_u32\": %.1f, \"v_add3_u32\": %.1f, "
                "\"v_alignbyte_b32\": %.1f, \"v_perm_b32\": %.1f, \"v_pk_add_u16\": %.1f, "
                "\"v_add_u32_sdwa\": %.1f, \"v_add_f32\": %.1f, \"v_fma_f32\": %.1f, \"v_fma_mix_f32\": %.1f, "
                "\"v_add_f64\": %.1f, \"v_max_f64\": %.1f}, "
                "\"hbm_copy_bytes_per_s\": %.4e, "
                "\"hbm_copy_inflight_bytes_per_s\": %.4e, \"hbm_copy_inflight_loads_per_thread\": %d, "
                "\"hbm_copy_inflight_workgroups_per_cu\": %d, "
                "\"hbm_read_bytes_per_s\": %.4e, \"hbm_read_loads_per_thread\": %d, \"hbm_read_workgroups_per_cu\": %d}\n",
                prop.name, cus, clk_hz / 1e6, add32, add16, perm_add, add32 / cus / clk_hz, add16 / cus / clk_hz,
                lds_bw(t_l4, 4), lds_bw(t_l8, 8), lds_bw(t_l16, 16), lds_bw(t_l16, 16) / cus / clk_hz,
                lds_bw(t_l4, 4) / cus / clk_hz, v3_rate[0], v3_rate[1], v3_rate[2],
                lds_clk(t_l4, waves * lit * 8), lds_clk(t_l8, waves * lit * 8), lds_clk(t_l16, waves * lit * 8),
                lds_clk(t_s9, waves * lit * 4 * 5), lds_clk(t_ua, waves * uit * 4), lds_clk(t_r16o, waves * uit * 4),
                n_wrong, lds_clk(t_w4, waves * lit * 4), lds_clk(t_w8, waves * lit * 4), lds_clk(t_w16, waves * lit * 4),
                t_is[0], t_is[1], t_is[2], t_is[3], t_is[4], t_is[5], t_is[6], t_is[7], t_is[8], t_is[9], t_is[10], copy_bw,
                copy_u_bw, copy_u_best[0], copy_u_best[1], read_u_bw, read_u_best[0], read_u_best[1]);
    CHECK(hipFree(src));
    CHECK(hipFree(dst));
    CHECK(hipFree(in));
    CHECK(hipFree(out));
    return 0;
}
