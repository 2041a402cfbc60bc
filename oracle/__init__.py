"""CPU oracle for sub-band dedispersion and the boxcar matched filter.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything in this package.
Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP path.

It is a plain, slow, obviously correct restatement of what the paper
(Men & Barr, "TransientX: A high performance single pulse search package")
computes on its hot path:

* the cold-plasma delay (Sec. 2.3, Eq. 1) turned into integer sample delays;
* per-channel power sums, skewness and kurtosis, and the channel mask of the
  narrow-band RFI filter (Sec. 2.2);
* per-channel normalisation (Sec. 2.1: zero mean and unit variance, or
  inverse-variance weights), dedispersion of the normalised block and the
  matched filter of its float series;
* the "transpose" of time-major blocks into channel rows (Sec. 2.3,
  Fig. "dedispersion_flow");
* downsampling in time before a DM range of a dedispersion plan (Sec. 2.3);
* brute-force dedispersion (Sec. 2.3, the O(N_DM N_t N_f) method);
* two-stage sub-band dedispersion (Sec. 2.3: coarse DM grid per sub-band,
  then the fine DM grid over the sub-banded series; Fig. "subband");
* per-DM noise statistics and the boxcar S/N of Sec. 2.4, Eq. 5, computed
  from a running sum and the difference of two of its values;
* the DM-time plane: best width per (DM, time), thresholded (Sec. 2.5);
* DBSCAN clustering of that plane with DM turned into delay (Sec. 2.5).

Where the paper is silent (the dispersion constant's value, the reference
frequency, rounding of delays, how the coarse grid is chosen, the boxcar
window for even widths, the noise estimator) the functions say which reading
they take.

Integer work is exact (int64).  Floating point is IEEE float64 evaluated in the
order written, with no fused multiply-add.
"""

from .ref import (  # noqa: F401
    K_DM,
    delay_samples,
    Plan,
    make_plan,
    group_size_rule,
    channel_rows,
    downsample,
    dedisperse_brute,
    subband_stage1,
    subband_stage2,
    dedisperse_subband,
    dedisperse_offsets,
    dm_stats,
    snr_from_sum,
    boxcar_snr_series,
    boxcar_peak,
    boxcar_peaks,
    boxcar_candidates,
    boxcar_snr_fixed,
    delay_axis,
    dbscan_plane,
    channel_power_sums,
    channel_moments,
    skf_mask,
    WEIGHT_UNIT,
    WEIGHT_INVERSE_VAR,
    channel_mean_var,
    norm_weights,
    normalise,
    dedisperse_subband_norm,
    norm_abs_bound,
    float_stats,
    boxcar_snr_series_float,
    boxcar_peaks_float,
    boxcar_candidates_float,
)
