/*
 * libtx: two-stage sub-band incoherent dedispersion of uint8 filterbank blocks
 * and the boxcar matched filter, on AMD Instinct MI355X (gfx950).
 *
 * The operations follow Men & Barr, "TransientX: A high performance single
 * pulse search package":
 *   - cold-plasma delay, Sec. 2.3 Eq. 1;
 *   - sub-band dedispersion, Sec. 2.3 (coarse DM grid per sub-band, then the
 *     fine grid over the sub-banded series) and Fig. "subband";
 *   - block processing with a carried-over tail ("shift data"), Sec. 2.3 and
 *     Fig. "dedispersion_flow";
 *   - boxcar S/N from a running sum, Sec. 2.4 Eq. 5;
 *   - the thresholded DM-time plane (best width per DM and time), Sec. 2.5.
 *
 * Conventions for every call:
 *   - Every call returns a tx_status; 0 is success.  Nothing throws across the
 *     ABI.  Errors from work already queued on a stream surface as TX_EDEVICE
 *     on a later call that synchronises, or from the caller's own stream sync.
 *   - "d_" pointers are device memory on the current HIP device; "host_"
 *     pointers are host memory.  The caller owns every buffer it passes;
 *     no call frees caller memory.  Plans, streams and batches own their
 *     tables, rings and scratch and release them in the matching destroy call.
 *   - Device work is queued on the given hipStream_t (0 = the null stream) and
 *     is asynchronous unless stated otherwise.
 *   - Plans are immutable after creation and may be shared between threads and
 *     streams.  Streams and batches have a single owner.
 */
#ifndef TX_H
#define TX_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tx_status {
    TX_OK = 0,
    TX_EINVAL = -1,     /* an argument is out of range or inconsistent */
    TX_ENOMEM = -2,     /* host or device allocation failed */
    TX_EDEVICE = -3,    /* a HIP runtime call failed (no device, launch error, fault) */
    TX_ESTATE = -4,     /* the object is not in a state that allows this call */
    TX_EOVERFLOW = -5,  /* a delay or size does not fit the exact integer path */
    TX_ENOTSUP = -6     /* the call is valid but the library does not support it */
} tx_status;

/* Human-readable name of a status code.  Never NULL. */
const char* tx_status_str(tx_status s);

/* Return the stream-ordered scratch that libtx calls have freed on the
 * current device to the system (libtx keeps it pooled for reuse otherwise).
 * Synchronises the device.  Errors: TX_EDEVICE. */
tx_status tx_pool_trim(void);

/* Version string of the library build. */
const char* tx_version(void);

/* Text of the last HIP runtime error that made a call on this thread return
 * TX_EDEVICE or TX_ENOMEM, or of the reason tx_dedisperse_noalloc returned
 * TX_ENOTSUP ("" if none).  Owned by the library. */
const char* tx_last_error(void);

/* ------------------------------------------------------------------------ */
/* Plans (Sec. 2.3)                                                          */
/* ------------------------------------------------------------------------ */

typedef struct tx_plan_s* tx_plan_t;

/* Flags for tx_plan_ex. */
#define TX_PLAN_HOST_ONLY 1u   /* build the host tables only; no device upload */

/*
 * tx_plan: build a dedispersion plan.
 *
 *   freqs_mhz[nchan]  channel centre frequencies in MHz, any order; channel
 *                     c of every input block is row c.  Finite and > 0.
 *   tsamp_s           sampling interval in seconds, finite and > 0.
 *   dms[ndm]          fine DM trials in pc cm^-3, finite, >= 0, non-decreasing.
 *   nsub              number of sub-bands; must divide nchan, and
 *                     nchan / nsub <= 256 (the first stage sums up to 256
 *                     uint8 channels exactly in 16 bits).  0 asks the plan to
 *                     pick nsub itself (the divisor of nchan with at most 256
 *                     channels per sub-band that minimises N_c * nchan +
 *                     2.5 * ndm * nsub, the additions per output sample of
 *                     the two stages weighted by their cost on MI355X).
 *
 * Delays follow Sec. 2.3 Eq. 1 with k = 4.148808e3 s MHz^2 pc^-1 cm^3:
 *   D(DM, f) = floor(((k*DM) * (1/(f*f) - 1/(fref*fref))) / tsamp + 0.5),
 * evaluated on the host in IEEE float64 in that order, fref = the highest
 * channel frequency.  Sub-band s is the run of nchan/nsub contiguous channels
 * starting at s*nchan/nsub; its reference frequency is its highest channel.
 * The fine trials are cut into consecutive groups of g; a group's coarse DM is
 * its first trial.  g = 1 + floor((a_full / a_max) / 2), capped at ndm, where
 * a = 1/f_lo^2 - 1/f_hi^2 over the whole band (a_full) and over the widest
 * sub-band (a_max): the coarse-DM error inside a sub-band then stays within
 * the full-band delay change of half a fine DM step.  With one channel per
 * sub-band, g = ndm (exact).
 *
 * The plan's tables are uploaded to the current device.  On success *out
 * holds a new plan that the caller releases with tx_plan_destroy.
 * Errors: TX_EINVAL (bad argument), TX_EOVERFLOW (a delay >= 2^30 samples),
 * TX_ENOMEM, TX_EDEVICE (no usable device or upload failed).
 */
tx_status tx_plan(const double* freqs_mhz, int32_t nchan, double tsamp_s,
                  const double* dms, int32_t ndm, int32_t nsub, tx_plan_t* out);

/*
 * tx_plan_ex: tx_plan with two overrides.
 *   dms_per_group  0 = the rule above; otherwise g itself (1 gives brute
 *                  force: every trial is its own coarse DM).  Clamped to ndm.
 *   flags          TX_PLAN_HOST_ONLY builds the host tables without touching
 *                  any device (such a plan answers queries only; device calls
 *                  on it return TX_ESTATE).
 */
tx_status tx_plan_ex(const double* freqs_mhz, int32_t nchan, double tsamp_s,
                     const double* dms, int32_t ndm, int32_t nsub,
                     int32_t dms_per_group, uint32_t flags, tx_plan_t* out);

typedef struct tx_plan_info {
    int32_t nchan;        /* channels */
    int32_t ndm;          /* fine DM trials */
    int32_t nsub;         /* sub-bands (after the automatic choice) */
    int32_t chans_per_sub;/* nchan / nsub */
    int32_t g;            /* fine trials per coarse group */
    int32_t ngroups;      /* coarse groups = ceil(ndm / g) */
    int64_t overlap;      /* O: input samples needed beyond the output length */
    int64_t max_extent;   /* largest extra length of a first-stage series */
    int64_t brute_reach;  /* D(max DM, lowest frequency) */
    double fref_mhz;      /* reference frequency (highest channel) */
    double tsamp_s;
    int32_t on_device;    /* 1 if the tables live on a device */
    int32_t device;       /* that device's ordinal, or -1 */
} tx_plan_info;

/* Fill *info.  Errors: TX_EINVAL on NULL arguments. */
tx_status tx_plan_query(tx_plan_t plan, tx_plan_info* info);

/*
 * Effective per-(trial, channel) offsets host_off[ndm * nchan] (row-major by
 * trial):  off(i, ch) = D(c_j, f_ch) + D(dm_i, f_s) - D(c_j, f_s), with j the
 * group of trial i and s the sub-band of ch.  The two stages compute exactly
 * Y[i][t] = sum over ch of x[ch][t + off(i, ch)].  Host memory, caller-owned.
 */
tx_status tx_plan_offsets(tx_plan_t plan, int32_t* host_off);

/*
 * Host copies of the plan tables; any pointer may be NULL.
 *   coarse_chan[ngroups * nchan] = D(c_j, f_ch)
 *   coarse_sub [ngroups * nsub]  = D(c_j, f_s)
 *   fine_sub   [ndm * nsub]      = D(dm_i, f_s)
 *   extent     [ngroups * nsub]  = max over i in j of D(dm_i, f_s) - D(c_j, f_s)
 */
tx_status tx_plan_tables(tx_plan_t plan, int32_t* coarse_chan, int32_t* coarse_sub,
                         int32_t* fine_sub, int32_t* extent);

/* Brute-force delays host_delay[nchan] = D(dm, f_ch) for one DM (>= 0). */
tx_status tx_plan_delays(tx_plan_t plan, double dm, int32_t* host_delay);

/* Release a plan.  The caller must not use it afterwards, nor destroy it while
 * device work that uses it is still queued.  NULL is accepted. */
tx_status tx_plan_destroy(tx_plan_t plan);

/* ------------------------------------------------------------------------ */
/* Stateless dedispersion (Sec. 2.3)                                         */
/* ------------------------------------------------------------------------ */

/*
 * Bytes of device scratch that tx_dedisperse_ws needs for output length nt
 * (the first-stage series of every coarse group and sub-band, uint16).
 * TX_ENOTSUP, as tx_dedisperse answers it, when a staged row of the plan's
 * tiles does not fit the device's LDS (a group of trials spanning a very
 * wide range of delays).
 */
tx_status tx_dedisperse_ws_size(tx_plan_t plan, int64_t nt, int64_t* bytes);

/*
 * tx_dedisperse: Y = two-stage sub-band dedispersion of one block.
 *
 *   d_in      uint8, nchan rows; row c starts at d_in + c*in_pitch and holds
 *             at least nt + overlap valid samples (overlap from
 *             tx_plan_query).  d_in and in_pitch must be multiples of 16.
 *   nt        output samples per trial, >= 0 (0 queues nothing).
 *   d_out     int32, ndm rows; row i starts at d_out + i*out_pitch elements
 *             (out_pitch >= nt, a multiple of 2; d_out 8-byte aligned).
 *             Y[i][t] = sum over s of B[j][s][t + D(dm_i,f_s) - D(c_j,f_s)],
 *             B[j][s][u] = sum over ch in s of x[ch][u + D(c_j, f_ch)].
 *   stream    HIP stream for all work.
 *
 * Every value is an exact integer sum (bit-exact for any tiling).  Scratch for
 * the first stage comes from the device's stream-ordered memory pool and is
 * returned to it on the same stream.
 * Errors: TX_EINVAL, TX_ESTATE (host-only plan or another device current),
 * TX_ENOMEM, TX_EDEVICE.
 */
tx_status tx_dedisperse(tx_plan_t plan, const uint8_t* d_in, int64_t in_pitch, int64_t nt,
                        int32_t* d_out, int64_t out_pitch, hipStream_t stream);

/* tx_dedisperse with caller-provided scratch d_ws of ws_bytes bytes
 * (>= tx_dedisperse_ws_size, 256-byte aligned).  The scratch must not be used
 * by other work on any stream until this call's work has finished. */
tx_status tx_dedisperse_ws(tx_plan_t plan, const uint8_t* d_in, int64_t in_pitch, int64_t nt,
                           int32_t* d_out, int64_t out_pitch, void* d_ws, int64_t ws_bytes,
                           hipStream_t stream);

/*
 * tx_dedisperse_noalloc: tx_dedisperse for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation during a run).  Same arguments, layout, result and
 * errors as tx_dedisperse; it calls no allocator.  The first-stage series go
 * to a scratch array of TX_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends, and the block is processed in
 * chunks of output samples whose series fit it (so a large block takes
 * several launches of each stage; the plan's first-stage tile may be swapped
 * for a shorter one, which changes no result).  All calls on one GPU share
 * that array: calls that overlap on one GPU (on other streams or threads)
 * race and give wrong results; calls queued on one stream are ordered.
 * Errors: those of tx_dedisperse, and TX_ENOTSUP when one chunk of the
 * plan's series does not fit the array (tx_last_error gives the bytes it
 * would need).
 */
#define TX_NOALLOC_SCRATCH_BYTES (256ll << 20)
tx_status tx_dedisperse_noalloc(tx_plan_t plan, const uint8_t* d_in, int64_t in_pitch, int64_t nt,
                                int32_t* d_out, int64_t out_pitch, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Time-major ingest (Sec. 2.3, Fig. "dedispersion_flow", "transpose" step)  */
/* ------------------------------------------------------------------------ */

/*
 * tx_transpose_tf: channel rows from a time-major block, as recorded (one
 * row of nchan channel bytes per time sample).
 *
 *   d_tf      uint8, nt rows; row t starts at d_tf + t*tf_pitch and holds the
 *             nchan channel samples of time t (tf_pitch >= nchan).
 *   d_ft      uint8, nchan rows; row c starts at d_ft + c*ft_pitch and
 *             receives d_ft[c][t] = d_tf[t][c] for t < nt (ft_pitch >= nt);
 *             bytes past nt are untouched.
 *   d_tf, d_ft, tf_pitch and ft_pitch must be multiples of 16.
 *
 * Pure data movement (every byte read and written once), asynchronous on
 * `stream`.  Errors: TX_EINVAL, TX_EDEVICE.
 */
tx_status tx_transpose_tf(const uint8_t* d_tf, int64_t tf_pitch, int32_t nchan, int64_t nt, uint8_t* d_ft,
                          int64_t ft_pitch, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Channel masks (Sec. 2.2, narrow-band RFI removal)                          */
/* ------------------------------------------------------------------------ */

/*
 * Drop channels from a plan's sums: mask[c] == 0 gives channel c weight 0 in
 * every trial of every later dedispersion with this plan (its samples are
 * read as zeros), exactly as if its row were zero; non-zero keeps it.  NULL,
 * or a mask that keeps every channel, removes the mask.  Waits for all queued
 * device work first (queued work may read the mask).  Errors: TX_EINVAL,
 * TX_ESTATE (host-only plan), TX_ENOMEM, TX_EDEVICE.
 */
tx_status tx_plan_set_mask(tx_plan_t plan, const uint8_t* mask);
/* The plan's mask as nchan bytes of 0 / 1 (all 1 without a mask). */
tx_status tx_plan_get_mask(tx_plan_t plan, uint8_t* mask);

/*
 * tx_channel_power_sums: d_sums[4c + j] = sum over t < nt of x[c][t]^(j+1),
 * j = 0..3, exact in uint64, for the nchan channel rows of d_in (row c at
 * d_in + c*in_pitch; d_in and in_pitch multiples of 16, in_pitch >= nt,
 * nt <= 2^32; d_sums 8-byte aligned, 4*nchan values).  Asynchronous on
 * `stream`.  Errors: TX_EINVAL, TX_EDEVICE.
 */
tx_status tx_channel_power_sums(const uint8_t* d_in, int64_t in_pitch, int32_t nchan, int64_t nt, uint64_t* d_sums,
                                hipStream_t stream);

/*
 * tx_skf_mask (host): the skewness-kurtosis channel mask from power sums of
 * nt samples per channel (host array, 4*nchan values; 1 <= nt <= 2^23).
 * Per channel, from exact integer central moments: skewness m3 / m2^1.5 and
 * kurtosis m4 / m2^2.  Over the channels with m2 > 0, a channel is an outlier
 * in a statistic when its distance to the median exceeds threshold times
 * 1.482602218505602 times the median absolute deviation (with a zero
 * deviation, any value off the median).  mask[c] = 0 for outliers in either
 * statistic and for channels with m2 = 0, else 1.  Errors: TX_EINVAL.
 */
tx_status tx_skf_mask(const uint64_t* sums, int32_t nchan, int64_t nt, double threshold, uint8_t* mask);

/* ------------------------------------------------------------------------ */
/* Normalisation (Sec. 2.1) and the floating-point variant of the path        */
/* ------------------------------------------------------------------------ */

#define TX_WEIGHT_UNIT 0          /* scale by 1/sigma: zero mean, unit variance per channel */
#define TX_WEIGHT_INVERSE_VAR 1   /* scale by 1/sigma^2: inverse-variance weights */

/*
 * tx_norm_weights (host): per-channel normalisation (Sec. 2.1) from exact
 * power sums of nt samples per channel (host array, 4*nchan values as
 * tx_channel_power_sums writes them; 1 <= nt <= 2^32).  Per channel the mean
 * S1/n and the population variance (n S2 - S1^2)/n^2 (exact integer
 * numerator, one rounding to float64); a normalised sample is
 * scale[c] * x - offset[c] with
 *   TX_WEIGHT_UNIT:        scale = 1/sigma,   offset = mean/sigma
 *                          (zero mean and unit variance in every channel);
 *   TX_WEIGHT_INVERSE_VAR: scale = 1/sigma^2, offset = mean/sigma^2
 *                          (each channel weighted by its inverse variance),
 * computed in float64 and rounded to float32 once.  A channel of zero
 * variance gets scale = offset = 0 (it adds nothing).  scale, offset: host
 * arrays of nchan floats.  Errors: TX_EINVAL (bad argument, or sums that
 * cannot belong to one channel).
 */
tx_status tx_norm_weights(const uint64_t* sums, int32_t nchan, int64_t nt, int32_t weighting, float* scale,
                          float* offset);

/*
 * tx_dedisperse_norm: two-stage sub-band dedispersion of the normalised block
 * (Sec. 2.1 then Sec. 2.3), in float32.  Arguments as tx_dedisperse, plus
 * d_scale, d_offset (device float[nchan], 4-byte aligned): channel c's sample
 * x enters as scale[c] * x - offset[c], rounded to float32 once (a fused
 * multiply-add); d_out is float32, ndm rows of out_pitch elements (>= nt,
 * 4-byte aligned).  Y[i][t] = sum over s of B[j][s][t + D(dm_i,f_s) -
 * D(c_j,f_s)], B[j][s][u] = sum over ch in s of the normalised samples at
 * u + D(c_j, f_ch) (the plan's offsets).  Summed in float32 in that order, a
 * value differs from the exact sum by at most (m + nsub + 1) * 2^-24 times
 * the sum of the absolute normalised samples it adds (m = channels per
 * sub-band).  Scratch (4 bytes per first-stage sample) comes from the
 * device's stream-ordered pool.  The plan's channel mask and tiles do not
 * apply (a dropped channel is one with scale = offset = 0).  Errors:
 * TX_EINVAL, TX_ESTATE, TX_ENOMEM, TX_ENOTSUP (a staged row does not fit the
 * device's LDS), TX_EDEVICE.
 */
tx_status tx_dedisperse_norm(tx_plan_t plan, const uint8_t* d_in, int64_t in_pitch, int64_t nt,
                             const float* d_scale, const float* d_offset, float* d_out, int64_t out_pitch,
                             hipStream_t stream);
/* Bytes of scratch tx_dedisperse_norm takes from the pool for nt outputs. */
tx_status tx_dedisperse_norm_ws_size(tx_plan_t plan, int64_t nt, int64_t* bytes);

/* ------------------------------------------------------------------------ */
/* DM ranges with downsampling (Sec. 2.3, dedispersion plans)                 */
/* ------------------------------------------------------------------------ */

/*
 * tx_downsample: out[c][t] = (sum of in[c][k t + i] for i < k, + k/2) / k
 * (integer division: the mean of k consecutive samples rounded to nearest,
 * halves up) for c < nchan, t < nt_out; k a power of two, 1..64.
 *
 *   d_in      uint8, nchan rows, row c at d_in + c*in_pitch, >= k*nt_out
 *             samples (in_pitch >= k*nt_out).
 *   d_out     uint8, nchan rows, row c at d_out + c*out_pitch (>= nt_out).
 *   Pointers and pitches must be multiples of 16.
 *
 * Bound by HBM (k + 1 bytes per output).  Errors: TX_EINVAL, TX_EDEVICE.
 */
tx_status tx_downsample(const uint8_t* d_in, int64_t in_pitch, int32_t nchan, int64_t nt_out, int32_t k,
                        uint8_t* d_out, int64_t out_pitch, hipStream_t stream);

/*
 * A dedispersion plan in DM ranges: range r dedisperses the block
 * downsampled by factors[r] (tx_downsample) with plans[r], a plan over the
 * same channels at sampling time tsamp * factors[r] (tsamp the block's own),
 * typically covering a higher DM range with a coarser DM step.  The plans
 * are borrowed: they must outlive the ranges object.  n is 1..64, every
 * factor a power of two, 1..64.  Errors: TX_EINVAL (factor, channels or
 * sampling times inconsistent), TX_ESTATE (host-only plan, or plans on
 * different devices), TX_ENOMEM.
 */
typedef struct tx_ranges_s* tx_ranges_t;
tx_status tx_ranges_create(const tx_plan_t* plans, const int32_t* factors, int32_t n, tx_ranges_t* out);

/* Input samples per channel that a block of nt full-rate samples needs: the
 * largest factors[r] * (nt / factors[r] + overlap_r).  nt must be a multiple
 * of every factor (else TX_EINVAL). */
tx_status tx_ranges_input_len(tx_ranges_t r, int64_t nt, int64_t* need);

/*
 * Dedisperse one block in every range.  d_in as for tx_dedisperse, with
 * in_pitch >= tx_ranges_input_len(nt).  Range r writes plans[r]'s ndm rows of
 * nt / factors[r] samples to d_outs[r] (out_pitches[r] elements per row, as
 * for tx_dedisperse).  Each distinct factor > 1 downsamples the block once
 * into a buffer from the device's stream-ordered pool, returned on `stream`.
 * Every output equals tx_dedisperse of plans[r] on tx_downsample's output.
 * Errors: TX_EINVAL, TX_ESTATE, TX_ENOMEM, TX_ENOTSUP, TX_EDEVICE.
 */
tx_status tx_ranges_dedisperse(tx_ranges_t r, const uint8_t* d_in, int64_t in_pitch, int64_t nt,
                               int32_t* const* d_outs, const int64_t* out_pitches, hipStream_t stream);

/* Release a ranges object (not its plans).  NULL is accepted. */
tx_status tx_ranges_destroy(tx_ranges_t r);

/* ------------------------------------------------------------------------ */
/* Tile shapes (choices of the kernel implementation; results never change)  */
/* ------------------------------------------------------------------------ */

typedef struct tx_tiles {
    int32_t stage1;      /* first-stage variant, 0..count-1, or -1 for the library's default */
    int32_t stage1_lds;  /* LDS bytes per first-stage workgroup, 0 = default (raised
                            to what one staged row of the plan's widest channel
                            window plus the workgroup's shift tables need) */
    int32_t stage2;      /* second-stage variant, or -1 */
    int32_t stage2_lds;  /* LDS bytes per second-stage workgroup, 0 = default (raised
                            likewise for one sub-band row, both copies, and the
                            offset table) */
} tx_tiles;

/* Number of kernel variants of a stage (1 or 2). */
tx_status tx_tile_variants(int32_t stage, int32_t* count);

/* Shape of one variant: output samples per workgroup tile, and (stage 1) the
 * coarse trials each of the workgroup's 4 wavefronts accumulates. */
tx_status tx_tile_variant_info(int32_t stage, int32_t variant, int32_t* outputs_per_tile,
                               int32_t* trials_per_wave);

/* Read / replace the plan's tile choice.  Every choice gives bit-identical
 * output; only speed and scratch size change.  The setter is the one mutation
 * a plan allows: do not call it while device work using the plan is being
 * queued from another thread. */
tx_status tx_plan_get_tiles(tx_plan_t plan, tx_tiles* tiles);
tx_status tx_plan_set_tiles(tx_plan_t plan, const tx_tiles* tiles);

/* The tiles a dedispersion of nt outputs with this plan launches with: the
 * plan's choice with defaults resolved (variant indices >= 0, LDS bytes as
 * raised to what the staged rows need).  Launches nothing; TX_EINVAL for
 * nt < 0. */
tx_status tx_plan_resolved_tiles(tx_plan_t plan, int64_t nt, tx_tiles* tiles);

/*
 * Autotuner: time every first-stage variant with the default second stage,
 * then every second-stage variant with the fastest first stage, dedispersing
 * a scratch block of nt outputs of the plan's shape on `stream` (effort 0:
 * default LDS sizes; 1: instead the sizes that fit 7, 6, 5, 4 and 3
 * workgroups in a 160 KB CU: 23392, 27296, 32768, 40960 and 54608 bytes per
 * workgroup), and store
 * the fastest pair in the plan as tx_plan_set_tiles would.  Scratch comes
 * from the device's stream-ordered pool; the call synchronises `stream`
 * (not for use under graph capture).  *best_ms (may be NULL) receives the
 * measured time of one dedispersion with the chosen tiles.  Errors:
 * TX_EINVAL, TX_ESTATE (host-only plan or another device), TX_ENOMEM,
 * TX_EDEVICE, TX_ENOTSUP (no variant fits the device's LDS).
 */
tx_status tx_plan_autotune(tx_plan_t plan, int64_t nt, int32_t effort, double* best_ms, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Matched filter (Sec. 2.4) and DM-time candidates (Sec. 2.5)               */
/* ------------------------------------------------------------------------ */

/* One thresholded point of the DM-time plane. */
typedef struct tx_cand {
    int32_t dm_index;  /* row of the DM x time array */
    int32_t width;     /* boxcar width with the highest S/N at this point */
    int64_t time;      /* first sample of the boxcar window */
    double snr;        /* its S/N */
} tx_cand;

#define TX_MAX_WIDTHS 32
#define TX_MAX_WIDTH 1024
#define TX_MAX_NT_BOXCAR (1 << 20)
#define TX_MAX_VALUE (1 << 21)

/*
 * tx_boxcar_snr: peak boxcar S/N of every row of a DM x time array.
 *
 *   d_dmt     int32 rows, row d at d_dmt + d*pitch elements, nt valid values,
 *             each value in [0, 2^21) (any dedispersed block of <= 8224
 *             channels).  A row holding a value outside that range yields
 *             snr = NaN, width = -1, time = -1.
 *   ndm, nt   rows and samples per row; 1 <= nt <= 2^20.
 *   widths    HOST array of nw (1..32) strictly increasing widths in [1, 1024].
 *   d_snr, d_width, d_time  device outputs [ndm].
 *
 * Per row (Sec. 2.4 Eq. 5, readings stated): the window of width w starting at
 * t holds samples [t, t+w) and must lie inside the row; its sum S comes from
 * the running sum of the row (uint32, exact as a difference).  The noise
 * sigma is the population standard deviation of the row: c = floor(sum/nt),
 * Q = sum (y - c)^2, r = sum - nt*c, var = Q/nt - (r/nt)^2 in float64; then
 * snr = ((double)(nt*S - w*sum) * (1/(sigma*nt))) * (1/sqrt(w)).
 * For each width the earliest t with the largest S is taken; the width with
 * the largest S/N wins, ties to the smaller width.  A row with var <= 0, or
 * with every width > nt, gives (0.0, widths[0], 0).
 */
tx_status tx_boxcar_snr(const int32_t* d_dmt, int32_t ndm, int64_t nt, int64_t pitch,
                        const int32_t* widths, int32_t nw,
                        double* d_snr, int32_t* d_width, int64_t* d_time, hipStream_t stream);

/*
 * tx_candidates: the thresholded DM-time plane (Sec. 2.5).  For every row d
 * and start t, w* is the width with the highest S/N at t (ties to the smaller
 * width, only windows inside the row); (d, t, w*, snr) is emitted when
 * snr >= gamma.  Rows with var <= 0 emit nothing.  Inputs as tx_boxcar_snr;
 * gamma must be finite.
 *
 *   d_out[cap]   device array of records, in no particular order (sort by
 *                (dm_index, time) on the host for a canonical list).
 *   d_count      device int64: set to the total number of points found, even
 *                when it exceeds cap (only the first cap found are stored).
 *   d_snr, d_width, d_time  optional (NULL or all three): the per-row peaks
 *                of tx_boxcar_snr, computed in the same pass.
 */
tx_status tx_candidates(const int32_t* d_dmt, int32_t ndm, int64_t nt, int64_t pitch,
                        const int32_t* widths, int32_t nw, double gamma,
                        tx_cand* d_out, int64_t cap, int64_t* d_count,
                        double* d_snr, int32_t* d_width, int64_t* d_time, hipStream_t stream);

/*
 * tx_boxcar_snr_f32 / tx_candidates_f32: tx_boxcar_snr and tx_candidates for
 * a float32 DM x time array (Sec. 2.4 Eq. 5, Sec. 2.5), evaluated in float64:
 * per row the mean and population variance S2/T - (S1/T)^2 of its T values;
 * the window [t, t+w) inside the row has sum S (float64 running sums) and
 * snr = ((S - w * mean) / sigma) / sqrt(w).  Per width the largest S/N, at
 * the earliest start of the largest window sum (the S/N never decreases with
 * the sum; where two different sums round to the same S/N the start may be
 * the later one), across widths the largest (ties to the smaller width); a
 * row of zero variance gives (0.0, widths[0], 0) and no candidates.  Other
 * arguments, limits and errors as the integer calls (no value-range flag).
 */
tx_status tx_boxcar_snr_f32(const float* d_dmt, int32_t ndm, int64_t nt, int64_t pitch, const int32_t* widths,
                            int32_t nw, double* d_snr, int32_t* d_width, int64_t* d_time, hipStream_t stream);
tx_status tx_candidates_f32(const float* d_dmt, int32_t ndm, int64_t nt, int64_t pitch, const int32_t* widths,
                            int32_t nw, double gamma, tx_cand* d_out, int64_t cap, int64_t* d_count,
                            double* d_snr, int32_t* d_width, int64_t* d_time, hipStream_t stream);

/*
 * tx_boxcar_snr_fixed: tx_boxcar_snr_f32 with the noise mean and sigma given
 * (finite, sigma > 0) instead of estimated from each row: snr = ((S - w mean)
 * / sigma) / sqrt(w) (Sec. 2.4 Eq. 5).  For checks of Eq. 5 and of the
 * width-mismatch loss on noise-free pulses, and for series whose noise is
 * known (a normalised block's).  Errors: TX_EINVAL.
 */
tx_status tx_boxcar_snr_fixed(const float* d_dmt, int32_t ndm, int64_t nt, int64_t pitch, const int32_t* widths,
                              int32_t nw, double mean, double sigma, double* d_snr, int32_t* d_width,
                              int64_t* d_time, hipStream_t stream);

/*
 * tx_cluster: DBSCAN of thresholded DM-time points (Sec. 2.5) to remove
 * duplicate detections of one pulse.
 *
 *   plan       the plan whose DM trials the points index.  Each point is
 *              placed at (x, t): x the dispersion delay of its DM across the
 *              band, k DM (1/f_lo^2 - 1/f_hi^2) / tsamp in samples (Eq. 1,
 *              unrounded), t its start sample.
 *   d_cands    n device records (any order, e.g. from tx_candidates), with
 *              dm_index in [0, ndm) and time in [0, 2^32); other records are
 *              treated as noise.  n < 2^31 - 1.
 *   radius     r in samples (0 < r <= 1e6): neighbours are the other points
 *              at Euclidean distance <= r.
 *   min_pts    k >= 0: a core point has more than k neighbours.
 *   d_sorted   n device records: the points sorted by (dm_index, time).
 *   d_label    device int32[n]: cluster of d_sorted[i], or -1 for noise.
 *              Core points connected through core neighbours share a
 *              cluster; a non-core point within r of core points joins the
 *              cluster of the nearest one (ties: the first in sorted order);
 *              clusters are numbered 0.. in the order of their first core
 *              point.
 *   d_rep      device int64[n]: d_rep[c] for c < C is the sorted index of
 *              cluster c's highest-S/N point (ties: the first); -1 beyond C.
 *   d_nclusters  device int64: C.
 *
 * Results are unique for the given points (no dependence on input order or
 * thread timing).  Scratch comes from the device's stream-ordered pool; the
 * call waits for its own work on `stream` before returning (its host-built
 * delay tables are copied on that stream).
 * Errors: TX_EINVAL, TX_ESTATE, TX_ENOMEM, TX_EDEVICE.
 */
tx_status tx_cluster(tx_plan_t plan, const tx_cand* d_cands, int64_t n, double radius, int32_t min_pts,
                     tx_cand* d_sorted, int32_t* d_label, int64_t* d_rep, int64_t* d_nclusters, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Streams: a beam's consecutive blocks (Sec. 2.3, Fig. "dedispersion_flow") */
/* ------------------------------------------------------------------------ */

/*
 * A stream keeps, on the device, the last `overlap` samples of every channel
 * of one beam (the not-yet-dedispersed tail that the paper's "shift data" step
 * moves to the front of the buffer), so that consecutive blocks dedisperse
 * exactly as their concatenation would.  The first `overlap` samples pushed
 * only prime the stream; after that, a push of nt samples emits nt outputs,
 * and output index k (counted from the first emitted sample) is
 * Y[i][k] = sum over ch of x[ch][k + off(i, ch)] of the concatenated input.
 */
typedef struct tx_stream_s* tx_stream_t;

/* Open a stream for blocks of at most max_block samples.  Allocates one
 * device buffer of nchan rows of overlap + max_block bytes (plus up to 127
 * bytes so that the history always ends, and every block is written, at a
 * 128-byte aligned byte; rows rounded up to 256 bytes) on the plan's device.
 * Each push moves the kept history back by the block length (128-byte aligned
 * destination; the source is aligned when the block length is a multiple of
 * 128, which makes the device-to-device copies several times faster).  The
 * first-stage scratch of standalone
 * pushes (tx_dedisperse_ws_size(max_block)) comes from the device's
 * stream-ordered pool on the first push that emits output, and stream jobs of
 * a batch use the batch's scratch instead.  Errors: TX_EINVAL, TX_ESTATE
 * (host-only plan), TX_ENOMEM, TX_EDEVICE. */
tx_status tx_stream_open(tx_plan_t plan, int64_t max_block, tx_stream_t* out);

/*
 * Push nt (1..max_block) new samples of every channel.  block: nchan rows of
 * nt samples, row c at block + c*block_pitch; host memory (pinned for an
 * asynchronous copy) when block_on_device is 0, device memory otherwise.
 * Writes *nt_out output samples per trial to d_out (ndm rows, out_pitch
 * elements apart; out_pitch >= nt, even; 8-byte aligned) and sets *nt_out
 * (0 while priming).  The block may be reused once the stream's work on
 * `stream` has completed.  Errors: TX_EINVAL, TX_ENOMEM, TX_EDEVICE.
 */
tx_status tx_stream_push(tx_stream_t s, const uint8_t* block, int64_t block_pitch, int64_t nt,
                         int32_t block_on_device, int32_t* d_out, int64_t out_pitch, int64_t* nt_out,
                         hipStream_t stream);

/*
 * tx_stream_push for a time-major block: nt rows of the plan's nchan channel
 * bytes, row t at block + t*block_pitch (block_pitch >= nchan; a device block
 * and its pitch must be multiples of 16).  The block is transposed
 * (tx_transpose_tf) straight into the stream's buffer; a host block is first
 * copied to a device staging buffer of max_block x nchan bytes (rounded up to
 * 16), taken from the device's stream-ordered pool on the first such push and
 * kept until close.  Outputs, ordering and errors are those of
 * tx_stream_push.
 */
tx_status tx_stream_push_tf(tx_stream_t s, const uint8_t* block, int64_t block_pitch, int64_t nt,
                            int32_t block_on_device, int32_t* d_out, int64_t out_pitch, int64_t* nt_out,
                            hipStream_t stream);

/* Samples received and output samples emitted since open / reset. */
tx_status tx_stream_position(tx_stream_t s, int64_t* received, int64_t* emitted);

/* Forget the history: the next pushes prime the stream again. */
tx_status tx_stream_reset(tx_stream_t s);

/*
 * Checkpoint: copy the held history (nchan x held samples, held <= overlap)
 * to host_hist (row c at host_hist + c*held) and report held and the
 * position; tx_stream_restore loads such a snapshot into an open stream of
 * the same plan.  Both synchronise `stream`.
 */
tx_status tx_stream_snapshot(tx_stream_t s, uint8_t* host_hist, int64_t* held, int64_t* received,
                             int64_t* emitted, hipStream_t stream);
tx_status tx_stream_restore(tx_stream_t s, const uint8_t* host_hist, int64_t held, int64_t received,
                            int64_t emitted, hipStream_t stream);

/* Release a stream (after its queued work has finished).  NULL is accepted. */
tx_status tx_stream_close(tx_stream_t s);

/* ------------------------------------------------------------------------ */
/* Batches: many beams of uneven shape in one set of launches                */
/* ------------------------------------------------------------------------ */

/*
 * A batch holds up to max_jobs jobs.  A job is one block of one beam: its
 * plan (channels, DM grid, sample time and tile variants may differ between
 * jobs), its input (a device block, or a stream plus the next host/device
 * block), its DM x time output and, optionally, its boxcar peaks and
 * candidates.  tx_batch_launch runs persistent launches: the first stage of
 * every job (one launch per first-stage tile variant in use), then the second
 * stage (one launch per trials-per-workgroup and variant class in use), then
 * the boxcar of every job; each launch is a grid of as many workgroups as the
 * device holds at once, and its workgroups take tile after tile (row after
 * row) from work counters in device memory.  Each result is bit-identical to
 * the job run alone.  With TX_BATCH_GRAPH the launches are captured into a
 * HIP graph on the first launch and replayed afterwards; the job table and
 * work counters live in device memory and are uploaded before every replay,
 * so later launches may carry any number of other jobs, of any size, as long
 * as their kernel classes and LDS sizes are among those captured (else
 * TX_ESTATE before anything is queued; tx_batch_reserve adds classes to a
 * graph not yet captured).
 */
typedef struct tx_batch_s* tx_batch_t;

#define TX_BATCH_GRAPH 1u

tx_status tx_batch_create(int32_t max_jobs, uint32_t flags, tx_batch_t* out);

/* Remove all jobs (allocations are kept). */
tx_status tx_batch_clear(tx_batch_t b);

/* Boxcar part of a job (all device pointers; see tx_candidates).  widths is a
 * host array copied at add time; d_cands/d_count may be NULL for peaks only. */
typedef struct tx_batch_boxcar {
    const int32_t* widths;
    int32_t nw;
    double gamma;
    double* d_snr;
    int32_t* d_width;
    int64_t* d_time;
    tx_cand* d_cands;
    int64_t cap;
    int64_t* d_count;
} tx_batch_boxcar;

/* Add a job on a device block (as tx_dedisperse).  box may be NULL. */
tx_status tx_batch_add(tx_batch_t b, tx_plan_t plan, const uint8_t* d_in, int64_t in_pitch, int64_t nt,
                       int32_t* d_out, int64_t out_pitch, const tx_batch_boxcar* box);

/* Add a job that pushes the next block of a stream (as tx_stream_push); the
 * number of output samples is reported by tx_batch_stream_output after the
 * launch was queued.  A stream may appear at most once per batch. */
tx_status tx_batch_add_stream(tx_batch_t b, tx_stream_t s, const uint8_t* block, int64_t block_pitch, int64_t nt,
                              int32_t block_on_device, int32_t* d_out, int64_t out_pitch,
                              const tx_batch_boxcar* box);
/* tx_batch_add_stream for a time-major block (as tx_stream_push_tf). */
tx_status tx_batch_add_stream_tf(tx_batch_t b, tx_stream_t s, const uint8_t* block, int64_t block_pitch,
                                 int64_t nt, int32_t block_on_device, int32_t* d_out, int64_t out_pitch,
                                 const tx_batch_boxcar* box);
tx_status tx_batch_stream_output(tx_batch_t b, int32_t job, int64_t* nt_out);

/* Declare, before the first launch, that jobs may use `plan` with at most
 * max_nt output samples and at most nw boxcar widths (0: no boxcar): the
 * graph captured by the first launch then also holds that plan's kernel
 * classes and LDS sizes (with its tile variants at reservation time), so
 * later launches with its jobs replay without TX_ESTATE.  count (1..max_jobs)
 * is checked only: persistent grids hold any number of jobs.  Errors:
 * TX_EINVAL, TX_ESTATE (plan on another device), TX_ENOTSUP (a tile does not
 * fit the device's LDS). */
tx_status tx_batch_reserve(tx_batch_t b, tx_plan_t plan, int32_t nw, int64_t max_nt, int32_t count);

/* Queue all jobs on `stream`.  The job table is uploaded on `stream` and the
 * host call waits until the previous launch of this batch has consumed its
 * table, so consecutive launches of one batch (and the pushes of one stream)
 * must be queued on the same HIP stream or ordered by the caller.  Errors:
 * TX_EINVAL (no jobs), TX_ESTATE (a job does not fit a captured graph),
 * TX_ENOMEM, TX_EDEVICE. */
tx_status tx_batch_launch(tx_batch_t b, hipStream_t stream);

/* Completion of the batch's last launch (all its kernels, copies and stream
 * shifts): tx_batch_wait blocks the host until that work has finished and
 * returns TX_EDEVICE (text in tx_last_error) if the device reported an error
 * for it; tx_batch_query sets *done to 1 when it has finished, 0 while it
 * runs, without blocking.  Before the first launch both report completion.
 * Errors: TX_EINVAL, TX_EDEVICE. */
tx_status tx_batch_wait(tx_batch_t b);
tx_status tx_batch_query(tx_batch_t b, int32_t* done);

tx_status tx_batch_destroy(tx_batch_t b);

/* ------------------------------------------------------------------------ */
/* Kernel timing                                                             */
/* ------------------------------------------------------------------------ */

/* Kernels whose launches can be timed. */
typedef enum tx_kernel {
    TX_KERNEL_STAGE1 = 0,   /* first stage: sub-bands at the coarse DMs */
    TX_KERNEL_STAGE2 = 1,   /* second stage: fine DMs from the sub-band series */
    TX_KERNEL_BOXCAR = 2,   /* boxcar S/N, peaks and candidates */
    TX_KERNEL_TRANSPOSE = 3, /* time-major to channel-major ingest */
    TX_KERNEL_DOWNSAMPLE = 4, /* time downsampling of a DM range */
    TX_KERNEL_COUNT = 5
} tx_kernel;

/*
 * tx_profile_enable: when on != 0, every later kernel launch of libtx is
 * bracketed by two hipEvents recorded on the launch's own stream (process-wide
 * switch; adds two event records per launch).  Turning it off keeps what was
 * recorded.
 */
tx_status tx_profile_enable(int32_t on);

/*
 * tx_profile_collect: wait for the recorded events of one kernel, return the
 * summed elapsed time in milliseconds and the number of launches, and forget
 * them.  Host-blocking.  Errors: TX_EINVAL (bad kernel id or NULL), TX_EDEVICE.
 */
tx_status tx_profile_collect(int32_t kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* TX_H */
