// Internal declarations shared by the host plan code, the C ABI and the HIP
// kernels of libtx.  Not part of the public interface.
#pragma once

#include <cstdint>
#include <mutex>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/tx.h"

namespace tx {

constexpr double kDispersion = 4.148808e3;  // s MHz^2 pc^-1 cm^3 (Sec. 2.3, Eq. 1)
constexpr int kMaxChansPerSub = 256;        // 256 * 255 < 2^16: exact uint16 first stage
constexpr int64_t kMaxDelay = int64_t(1) << 30;

// ---------------------------------------------------------------------------
// Tile shapes.  Stage 1 (first stage): a wave covers 256*Q1 consecutive
// outputs of J1W coarse trials; a workgroup has 4 waves sharing one time tile.
// Stage 2: each of the 4 waves covers 128*Q2 consecutive outputs of every
// fine trial in the workgroup's chunk of one coarse group.
// ---------------------------------------------------------------------------
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int Q1 = 4;
constexpr int J1W = 4;
constexpr int TT1 = 256 * Q1;            // outputs per stage-1 tile
constexpr int J1 = J1W * kWaves;         // coarse trials per stage-1 workgroup
constexpr int Q2 = 2;
constexpr int TT2 = 128 * Q2 * kWaves;   // outputs per stage-2 tile
constexpr int kLdsBudget = 48 * 1024;    // bytes of LDS per workgroup for the staged rows

// Boxcar kernel.
constexpr int kBoxTile = 4096;           // window starts per tile (16 per thread)
constexpr int kBoxPer = kBoxTile / kThreads;

// ---------------------------------------------------------------------------
// Kernel arguments.
// ---------------------------------------------------------------------------
struct Stage1Args {
    const uint8_t* x;       // input rows
    int64_t x_pitch;        // bytes between rows
    int64_t x_len;          // valid samples per row (nt + overlap)
    uint16_t* B;            // first-stage series [ngroups][nsub][B_pitch]
    int64_t B_pitch;        // elements per series (multiple of TT1)
    const int32_t* dcc;     // [ngroups][nchan] D(c_j, f_ch)
    int32_t nchan, nsub, m, ngroups;
    int32_t n_jchunks;      // ceil(ngroups / J1)
    int32_t n_ttiles;       // B_pitch / TT1
    int32_t lds_row;        // bytes per staged channel row (multiple of 16)
    int32_t cchunk;         // channels staged per pass
};

struct Stage2Args {
    const uint16_t* B;
    int64_t B_pitch;
    int32_t* Y;             // [ndm][y_pitch]
    int64_t y_pitch;
    int64_t nt;
    const int32_t* rel;     // [ndm][nsub] D(dm_i, f_s) - D(c_j, f_s)
    int32_t ndm, nsub, g, ngroups;
    int32_t n_ichunks;      // ceil(g / I2)
    int32_t n_ttiles;       // ceil(nt / TT2)
    int32_t lds_row;        // uint16 elements per staged sub-band row (multiple of 8)
    int32_t schunk;         // sub-bands staged per pass
    int32_t flush;          // sub-bands summed in 16 bits before widening
};

struct BoxcarArgs {
    const int32_t* y;
    int64_t pitch;
    int32_t ndm;
    int32_t nt;
    int32_t nw;
    int32_t wmax;           // largest width <= nt (0 if none)
    int32_t widths[TX_MAX_WIDTHS];
    double rsw[TX_MAX_WIDTHS];   // 1 / sqrt(w), computed on the host
    double gamma;
    int32_t want_peaks;
    int32_t want_cands;
    double* snr;
    int32_t* width;
    int64_t* time;
    tx_cand* cands;
    int64_t cap;
    unsigned long long* count;
};

// ---------------------------------------------------------------------------
// Plan object.
// ---------------------------------------------------------------------------
struct Launch1 {            // stage-1 launch geometry for one output length
    int32_t lds_row, cchunk;
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
    int32_t spread1 = 0;               // max first-stage shift spread inside a stage-1 tile
    int32_t spread2 = 0;               // max second-stage shift spread inside a stage-2 tile
    int device = -1;
    bool on_device = false;
    int32_t* d_coarse_chan = nullptr;
    int32_t* d_rel = nullptr;
};

namespace tx {

// Host plan construction (tx_plan.cpp).
tx_status build_plan_host(const double* freqs, int32_t nchan, double tsamp, const double* dms,
                          int32_t ndm, int32_t nsub, int32_t dms_per_group, tx_plan_s* p);
int32_t delay_samples(double dm, double f, double fref, double tsamp);

// Launch helpers (tx_kernels.hip).
struct DedispGeom {
    int64_t B_pitch;        // uint16 elements per first-stage series
    int64_t ws_bytes;       // scratch bytes
    int32_t lds1_row, cchunk;
    int32_t lds2_row, schunk;
    int32_t n_ttiles1, n_ttiles2;
};
DedispGeom dedisp_geometry(const tx_plan_s* p, int64_t nt);
hipError_t launch_dedisperse(const tx_plan_s* p, const DedispGeom& geo, const uint8_t* d_in,
                             int64_t in_pitch, int64_t nt, int32_t* d_out, int64_t out_pitch,
                             uint16_t* d_B, hipStream_t stream);
hipError_t launch_boxcar(const BoxcarArgs& a, hipStream_t stream);

// Optional per-launch timing (tx_profile.cpp).  prof_begin returns -1 when
// profiling is off; otherwise a slot whose end is recorded by prof_end.
int prof_begin(int kernel, hipStream_t stream);
void prof_end(int slot, hipStream_t stream);

}  // namespace tx
