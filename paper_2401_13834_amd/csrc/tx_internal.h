// Internal declarations shared by the host plan code, the C ABI and the HIP
// kernels of libtx.  Not part of the public interface.
#pragma once

#include <cstdint>
#include <mutex>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/tx.h"

#if defined(__HIP__)
// Global address space.  Pointers read from device memory (the job tables of
// a batch) are generic to the compiler, which then emits flat loads and stores
// that also count against the LDS wait counter; casting them to this address
// space keeps the kernels on global_load / global_store.  (The host pass of a
// HIP source sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define TX_GLOBAL __attribute__((address_space(1)))
#else
#define TX_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ TX_GLOBAL T* to_global(T* p) {
    return (TX_GLOBAL T*)(p);
}

// Work items [0, total) of a persistent launch, taken one at a time by whole
// workgroups from 8 counters in device memory (zero at the launch), counter x
// handing out the x-th contiguous eighth of the items.  A workgroup starts
// with the eighth of its own XCD (workgroup ids are dealt to the 8 XCDs in
// turn), so neighbouring items, which read the same input rows, share an L2,
// then helps with the others.  Every workgroup leaves once all 8 are spent.
template <typename F>
__device__ __forceinline__ void for_each_claimed(int total, uint32_t* queue, F&& f) {
    __shared__ int s_claim;
    const int x0 = static_cast<int>(blockIdx.x) & 7;
    const int q = total >> 3, r = total & 7;
    for (int k = 0; k < 8; ++k) {
        const int x = (x0 + k) & 7;
        const int lo = x * q + (x < r ? x : r);
        const int n = q + (x < r ? 1 : 0);
        for (;;) {
            if (threadIdx.x == 0) s_claim = static_cast<int>(atomicAdd(queue + x, 1u));
            __syncthreads();
            // uniform (a scalar register): the job lookup and its arguments
            // then stay scalar too
            const int c = __builtin_amdgcn_readfirstlane(s_claim);
            __syncthreads();
            if (c >= n) break;
            f(lo + c);
            __syncthreads();
        }
    }
}

namespace tx {

__device__ __forceinline__ uint32_t align_b32(uint32_t hi, uint32_t lo, uint32_t nbytes) {
    return __builtin_amdgcn_alignbyte(hi, lo, nbytes);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// s_waitcnt operand for "vector memory count 0", other counters untouched
// (vmcnt bits 3:0 and 15:14 zero, expcnt 6:4 = 7, lgkmcnt 11:8 = 15).
constexpr int kWaitVm0 = 0x0F70;

// Word 3 of a raw (stride 0) buffer resource on gfx9-family parts: 32-bit
// data format, no swizzle, no thread-id offset.
constexpr int kRawBufferWord3 = 0x00020000;

__device__ __forceinline__ __attribute__((address_space(3))) void* to_lds(uint8_t* p) {
    return (__attribute__((address_space(3))) void*)(p);
}

// Consecutive workgroup ids are dealt round-robin to the 8 XCDs; give each XCD
// a contiguous range of tiles so that tiles sharing input rows share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int total) {
    const int nx = 8;
    const int x = bid % nx, k = bid / nx;
    const int q = total / nx, r = total % nx;
    return x * q + min(x, r) + k;
}

// Largest v over a workgroup of 256 threads (red: 4 ints of LDS).
__device__ __forceinline__ int block_max(int v, int* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    v = max(max(red[0], red[1]), max(red[2], red[3]));
    __syncthreads();
    return v;
}

}  // namespace tx
#endif

namespace tx {

constexpr double kDispersion = 4.148808e3;  // s MHz^2 pc^-1 cm^3 (Sec. 2.3, Eq. 1)
constexpr int kMaxChansPerSub = 256;        // 256 * 255 < 2^16: exact uint16 first stage
constexpr int64_t kMaxDelay = int64_t(1) << 30;

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kTablePad = 64;            // padding of the trial axis of the transposed tables
constexpr int kMaxLds = 160 * 1024;      // LDS per workgroup on gfx950

// Boxcar kernel.
constexpr int kBoxTile = 4096;           // window starts per tile (16 per thread)
constexpr int kBoxPer = kBoxTile / kThreads;

// ---------------------------------------------------------------------------
// Kernel arguments.
// ---------------------------------------------------------------------------
struct Stage1Args {
    const uint8_t* x;       // input rows (16-byte aligned)
    int64_t x_pitch;        // bytes between rows
    int64_t x_len;          // valid samples per row (nt + overlap), counted from x_off
    int32_t x_off;          // first sample of every row at byte x_off (0..15) from x
    const uint8_t* mask;    // per channel, 0 = dropped (staged as zeros); null = keep all
    uint16_t* B;            // first-stage series [ngroups][nsub][B_pitch]
    int64_t B_pitch;        // elements per series (multiple of the time tile)
    const int32_t* dT;      // [nchan][gpad] D(c_j, f_ch), trial axis padded with the last group
    int32_t gpad;
    int32_t nchan, nsub, m, ngroups;
    int32_t n_jchunks;      // coarse-trial chunks per sub-band
    int32_t n_ttiles;       // B_pitch / time tile
    int32_t lds_bytes;      // dynamic LDS per workgroup
};

struct Stage2Args {
    const uint16_t* B;
    int64_t B_pitch;
    int32_t* Y;             // [ndm][y_pitch]
    int64_t y_pitch;
    int64_t nt;
    const int32_t* rT;      // [nsub][dpad] D(dm_i, f_s) - D(c_j, f_s), trial axis padded
    int32_t dpad;
    int32_t ndm, nsub, g, ngroups;
    int32_t n_ichunks;      // fine-trial chunks per group
    int32_t n_ttiles;       // ceil(nt / time tile)
    int32_t lds_bytes;
    int32_t flush;          // sub-bands summed in 16 bits before widening
};

struct BoxcarArgs {
    const int32_t* y;
    int64_t pitch;
    int32_t ndm;
    int32_t nt;
    int32_t nw;             // widths given
    int32_t ne;             // widths <= nt (a prefix: widths increase)
    int32_t wmax;           // largest width <= nt (0 if none)
    int32_t w_first;        // widths[0] as given (reported when ne == 0)
    // widths[0..ne) and their 1/sqrt(w) (computed on the host), padded to
    // TX_MAX_WIDTHS with the last entry so that kernels sized for more widths
    // than ne repeat a width instead of branching
    int32_t widths[TX_MAX_WIDTHS];
    double rsw[TX_MAX_WIDTHS];
    double gamma;
    int32_t want_peaks;
    int32_t want_cands;
    int32_t tmax_ok;        // the launch's dynamic LDS holds this row's per-(tile, width) maxima
    double* snr;
    int32_t* width;
    int64_t* time;
    tx_cand* cands;
    int64_t cap;
    unsigned long long* count;
};

// Dedispersion of normalised data and the float matched filter
// (tx_kernels_norm.hip).  Stage 1: workgroups of 4 kNormJW coarse trials and
// 256 kNormQ outputs (4 kNormQ per lane); stage 2: kNormIW fine trials and
// kNormTT2 outputs (3 per lane).
constexpr int kNormJW = 2;                 // stage 1: coarse trials per wave (8 per workgroup)
constexpr int kNormQ = 5;                  // stage 1: output dwords per lane (20 outputs; odd)
constexpr int kNormIW = 16;
constexpr int kNormTT2 = 768;
// Default LDS per workgroup of the two stages: 20 KB lets 8 workgroups share
// a CU (the register limit of both kernels), which measured faster than
// fewer workgroups with larger or double-buffered staging rounds.
constexpr int kNormLds = 20 * 1024;        // stage 2
constexpr int kNormLds1 = 20 * 1024;       // stage 1

struct Stage1NormArgs {
    const uint8_t* x;       // input rows (16-byte aligned)
    int64_t x_pitch;
    int64_t x_len;          // valid samples per row (nt + overlap)
    const float* scale;     // [nchan] normalised sample = scale x - offset
    const float* offset;
    float* B;               // [ngroups][nsub][B_pitch]
    int64_t B_pitch;
    const int32_t* dT;
    int32_t gpad;
    int32_t nsub, m, ngroups;
    int32_t n_jchunks, n_ttiles;
    int32_t lds_bytes;
};

struct Stage2NormArgs {
    const float* B;
    int64_t B_pitch;
    float* Y;
    int64_t y_pitch;
    int64_t nt;
    const int32_t* rT;
    int32_t dpad;
    int32_t ndm, nsub, g, ngroups;
    int32_t n_ichunks, n_ttiles;
    int32_t lds_bytes;
};

struct BoxcarNormArgs {
    const float* y;
    int64_t pitch;
    int32_t ndm;
    int32_t nt;
    int32_t ne;             // widths <= nt
    int32_t wmax;
    int32_t w_first;
    int32_t widths[TX_MAX_WIDTHS];
    double rsw[TX_MAX_WIDTHS];
    double gamma;
    int32_t want_peaks;
    int32_t want_cands;
    int32_t fixed;          // 1: use fixed_mean / fixed_sigma instead of the row's statistics
    int32_t tmax_ok;        // the per-(tile, width) table fits the launch's dynamic LDS (set by the launcher)
    double fixed_mean, fixed_sigma;
    double* snr;
    int32_t* width;
    int64_t* time;
    tx_cand* cands;
    int64_t cap;
    unsigned long long* count;
};

struct NormGeom {
    int64_t B_pitch;        // floats per first-stage series
    int64_t ws_bytes;       // scratch bytes
    int32_t n_ttiles1, n_ttiles2, n_jchunks, n_ichunks;
    int32_t lds1, lds2;
    bool ok;
};

// Tile variants (tx_kernels_dedisp.hip).  Stage 1: Q1 consecutive dwords (odd Q1, 4 outputs each)
// per lane, JW coarse trials per wave, 4 waves sharing one time tile of
// 256*Q1 outputs.  Stage 2: Q2 dwords (2 outputs each) per lane, the 4 waves
// splitting a time tile of 512*Q2 outputs, IW fine trials per workgroup.
struct Stage1Variant {
    int q, jw;
};
struct Stage2Variant {
    int q;
};
int stage1_variant_count();
int stage2_variant_count();
Stage1Variant stage1_variant(int v);
Stage2Variant stage2_variant(int v);

struct Tiles {
    int32_t s1 = -1, s1_lds = 0, s2 = -1, s2_lds = 0;   // -1 / 0: defaults
};

}  // namespace tx

struct tx_plan_s {
    int32_t nchan = 0, ndm = 0, nsub = 0, m = 0, g = 0, ngroups = 0;
    double tsamp = 0, fref = 0;
    std::vector<double> freqs, dms;
    std::vector<int32_t> coarse_chan;  // [ngroups][nchan]
    std::vector<int32_t> coarse_sub;   // [ngroups][nsub]
    std::vector<int32_t> fine_sub;     // [ndm][nsub]
    std::vector<int32_t> extent;       // [ngroups][nsub]
    std::vector<int32_t> rel;          // [ndm][nsub] fine minus coarse sub-band delay
    int64_t overlap = 0, max_extent = 0, brute_reach = 0;
    int32_t gpad = 0, dpad = 0;
    std::vector<int32_t> dT;           // [nchan][gpad]
    std::vector<int32_t> rT;           // [nsub][dpad]
    int device = -1;
    bool on_device = false;
    int32_t* d_dT = nullptr;
    int32_t* d_rT = nullptr;
    uint8_t* d_mask = nullptr;         // per channel: 0 drops it from every sum (null: keep all)
    std::vector<uint8_t> mask;         // host copy (empty: keep all)
    mutable std::mutex mu;             // guards `tiles` and the spread cache
    tx::Tiles tiles;
    mutable std::vector<std::pair<int, int32_t>> spread1_cache;   // (J, spread)
    mutable std::vector<std::pair<int, int32_t>> spread2_cache;   // (IW, spread)
};

struct tx_stream_s {
    tx_plan_s* plan = nullptr;
    int device = -1;
    int64_t max_block = 0;
    int64_t pitch = 0;                 // bytes per ring row (multiple of 256)
    // Ring row layout: [pad | history | new block].  The history always ends
    // at byte pad + overlap, a multiple of 128, so every block is written at a
    // cache-line boundary and the history occupies [pad + overlap - held, pad + overlap).
    uint8_t* ring = nullptr;
    int64_t pad = 0;                   // (128 - overlap % 128) % 128
    int64_t held = 0;                  // valid history samples of every row
    int64_t received = 0, emitted = 0;
    void* ws = nullptr;                // dedispersion scratch of standalone pushes (allocated on first use)
    int64_t ws_bytes = 0;
    uint8_t* stage = nullptr;          // device copy of a time-major host block (allocated on first use)
    int64_t stage_pitch = 0;           // bytes per staged time row (nchan rounded up to 16)
};

namespace tx {

// Stream steps shared by tx_stream_push and batches (tx_stream.cpp): copy a
// block behind the held history and report the outputs it completes; after
// those outputs were computed, keep only the last `overlap` samples.
tx_status stream_ingest(tx_stream_s* s, const uint8_t* block, int64_t block_pitch, int64_t nt, int block_on_device,
                        hipStream_t st, int64_t* n_out);
tx_status stream_advance(tx_stream_s* s, int64_t nt, hipStream_t st);
// As stream_ingest, for a time-major block (nt rows of nchan channel bytes):
// transposed into the stream's buffer, through the stream's staging buffer
// when the block is in host memory.
tx_status stream_ingest_tf(tx_stream_s* s, const uint8_t* block, int64_t block_pitch, int64_t nt,
                           int block_on_device, hipStream_t st, int64_t* n_out);
// First history sample of every row: the 16-byte aligned base and the byte
// offset (0..15) of that sample from it.
void stream_input(const tx_stream_s* s, const uint8_t** base, int* x_off);
tx_status check_out_args(const int32_t* d_out, int64_t out_pitch, int64_t nt);
// Validate a width list and fill widths, 1/sqrt(w), nw and the longest width <= nt.
tx_status boxcar_widths(const int32_t* widths, int32_t nw, int64_t nt, BoxcarArgs* a);
// Effective widths of a row of nt samples (ne, wmax and padding, from the
// widths given); call after boxcar_widths and whenever nt changes.
void boxcar_fit(BoxcarArgs* a, const int32_t* widths, int32_t nw, int64_t nt);
// Widths a boxcar kernel instance handles (4, 8, 10, 12, 16 or 32) for n widths.
int boxcar_nwt(int n);
tx_status status_of(hipError_t e);
// Keep freed stream-ordered scratch in the device's pool (idempotent per device).
tx_status retain_pool(int dev);
tx::Tiles plan_tiles(const tx_plan_s* p);

// Host plan construction (tx_plan.cpp).
tx_status build_plan_host(const double* freqs, int32_t nchan, double tsamp, const double* dms,
                          int32_t ndm, int32_t nsub, int32_t dms_per_group, tx_plan_s* p);
int32_t delay_samples(double dm, double f, double fref, double tsamp);
int32_t plan_spread1(const tx_plan_s* p, int J);    // largest D(c_j,f) - D(c_j0,f) within J trials
int32_t plan_spread2(const tx_plan_s* p, int iw);   // largest rel spread within iw fine trials

// Launch helpers (tx_kernels_dedisp.hip, tx_kernels_boxcar.hip).
struct DedispGeom {
    Tiles tiles;            // resolved variants and LDS sizes
    int tt1, J1, tt2, iw;
    int64_t B_pitch;        // uint16 elements per first-stage series
    int64_t ws_bytes;       // scratch bytes
    int32_t n_ttiles1, n_ttiles2, n_jchunks, n_ichunks;
    int32_t lds1, lds2;     // dynamic LDS per workgroup
    bool ok;                // false if some workgroup cannot fit its LDS rows
};
DedispGeom dedisp_geometry(const tx_plan_s* p, int64_t nt, const Tiles& want);
// Time-major [nt][tf_pitch] -> channel-major [nchan][ft_pitch] uint8
// (tx_kernels_transpose.hip); pointers and pitches multiples of 16.
hipError_t launch_transpose_tf(const uint8_t* d_tf, int64_t tf_pitch, int32_t nchan, int64_t nt, uint8_t* d_ft,
                               int64_t ft_pitch, hipStream_t stream);
// out[c][t] = rounded mean of in[c][k t .. k t + k - 1], t < nt_out, k a power
// of two up to 64 (tx_kernels_downsample.hip); pointers and pitches multiples
// of 16, in_pitch >= k * nt_out.
// DBSCAN of n DM-time points (tx_kernels_cluster.hip): d_x[ndm] delays in
// samples, [d_dlo[d], d_dhi[d]] the DM indices within the radius of d.
hipError_t launch_cluster(const tx_cand* d_in, int64_t n, int32_t ndm, const double* d_x, const int32_t* d_dlo,
                          const int32_t* d_dhi, double r, int32_t kmin, tx_cand* d_sorted, int32_t* d_label,
                          int64_t* d_rep, int64_t* d_nclusters, hipStream_t st);
// Exact per-channel (sum x, x^2, x^3, x^4) of nt samples (tx_kernels_stats.hip).
hipError_t launch_power_sums(const uint8_t* d_in, int64_t in_pitch, int32_t nchan, int64_t nt, uint64_t* d_sums,
                             hipStream_t stream);
hipError_t launch_downsample(const uint8_t* d_in, int64_t in_pitch, int32_t nchan, int64_t nt_out, int32_t k,
                             uint8_t* d_out, int64_t out_pitch, hipStream_t stream);
hipError_t launch_dedisperse(const tx_plan_s* p, const DedispGeom& geo, const uint8_t* d_in, int64_t in_pitch,
                             int64_t nt, int32_t* d_out, int64_t out_pitch, uint16_t* d_B, hipStream_t stream,
                             int x_off = 0);
hipError_t launch_boxcar(const BoxcarArgs& a, hipStream_t stream);
NormGeom norm_geometry(const tx_plan_s* p, int64_t nt);
hipError_t launch_dedisperse_norm(const tx_plan_s* p, const NormGeom& g, const uint8_t* d_in, int64_t in_pitch,
                                  int64_t nt, const float* scale, const float* offset, float* d_out,
                                  int64_t out_pitch, float* d_B, hipStream_t stream);
hipError_t launch_boxcar_norm(const BoxcarNormArgs& a, hipStream_t stream);
// tx_dedisperse_noalloc: chunks of the block through the file-scope scratch
// of device `dev` (current).  hipErrorInvalidValue with *need_bytes > 0 when
// one chunk's first-stage series do not fit it (the smallest need), -1 when
// no tile fits the device's LDS.
hipError_t launch_dedisperse_noalloc(const tx_plan_s* p, const Tiles& want, const uint8_t* d_in, int64_t in_pitch,
                                     int64_t nt, int32_t* d_out, int64_t out_pitch, hipStream_t stream, int dev,
                                     int64_t* need_bytes);

// Batch building blocks (tx_kernels_dedisp.hip, tx_kernels_boxcar.hip).
void fill_stage_args(const tx_plan_s* p, const DedispGeom& geo, const uint8_t* d_in, int64_t in_pitch, int64_t nt,
                     int32_t* d_out, int64_t out_pitch, uint16_t* d_B, Stage1Args* s1, Stage2Args* s2);
int64_t stage1_tiles(const Stage1Args& a);
int64_t stage2_tiles(const Stage2Args& a);
int stage2_iw(int32_t g);
// Device references of one batch launch (one kernel variant): its jobs start
// at jobs + info[1], their tile prefix sums at prefix + info[2] (info[0] + 1
// entries), info[0] jobs; queue holds the launch's 8 work counters.
struct BatchRefs {
    const void* jobs;
    const int* prefix;
    const int* info;
    uint32_t* queue;
};
// Persistent batch launches: as many workgroups as the device holds at once
// (fewer if `tiles` > 0 is smaller; 0 sizes a graph for any number of tiles).
hipError_t launch_stage1_batch(int variant, int lds, const BatchRefs& r, int64_t tiles, hipStream_t stream);
hipError_t launch_stage2_batch(int iw, int variant, int lds, const BatchRefs& r, int64_t tiles, hipStream_t stream);
// Boxcar over many row sets: rows of all jobs, job of a row by prefix sums.
hipError_t launch_boxcar_batch(int nwt, int lds, const BatchRefs& r, int64_t rows, hipStream_t stream);
// Workgroups of kernel `fn` the device holds at once with `lds` bytes of
// dynamic LDS (0 if unknown).
int resident_grid(const void* fn, int lds);
// Dynamic LDS bytes for the per-(tile, width) maxima of a row of nt samples
// with nwt widths, or 0 when they do not fit (the kernel then rescans every
// tile for candidates).
int boxcar_tmax_bytes(int nwt, int64_t nt);

hipError_t launch_zero_counts(const BoxcarArgs* d_jobs, const int* d_njobs, int max_jobs, hipStream_t stream);

// Largest dynamic LDS per workgroup the current device allows (capped at kMaxLds).
int device_max_lds();
// Last HIP error seen by the C ABI on this thread (tx_api.cpp).
void note_error(hipError_t e);
// Replace this thread's last-error text (tx_last_error) with a message.
void note_message(const char* msg);

// Optional per-launch timing (tx_profile.cpp).  prof_begin returns -1 when
// profiling is off; otherwise a slot whose end is recorded by prof_end.
int prof_begin(int kernel, hipStream_t stream);
void prof_end(int slot, hipStream_t stream);

}  // namespace tx
