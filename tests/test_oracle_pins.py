"""Pins of the CPU oracle to facts that the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints, closed forms, exact rational arithmetic, special cases that
reduce the method to brute force, invariants, and brute force on tiny inputs.
"""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        return json.load(f)


def _rand_plan(seed, nchan=32, nsub=8, ndm=23, f_top=1500.0, f_bot=1100.0, tsamp=1e-3, dm_max=300.0, g=None):
    rng = np.random.default_rng(seed)
    freqs = synth.band_centres(f_top, f_bot, nchan)
    dms = np.sort(rng.uniform(0.0, dm_max, ndm))
    dms[0] = 0.0
    return oracle.make_plan(freqs, tsamp, dms, nsub, g=g)


# ---------------------------------------------------------------------------
# The delay (Sec. 2.3, Eq. 1)
# ---------------------------------------------------------------------------

def test_dispersion_constant_matches_paper_zeta_coefficient():
    """Eq. 4's printed 6.91e-3 is 2 k sqrt(ln 2) with k in ms GHz^2: it fixes
    the dispersion constant to three digits."""
    z = _paper()["zeta_coefficient"]
    k_ms_ghz2 = oracle.K_DM * 1e3 / 1e6          # s MHz^2 -> ms GHz^2
    coeff = 2.0 * k_ms_ghz2 * 1e-3 * math.sqrt(math.log(2.0))   # per MHz of bandwidth
    assert float(f"{coeff:.{z['significant_digits']}g}") == pytest.approx(z["value"], rel=1e-12)


def test_dispersion_constant_from_physical_constants():
    """k = e^2 / (2 pi m_e c) in Gaussian units, converted to s MHz^2 pc^-1 cm^3."""
    e = 4.80320471e-10          # statcoulomb
    m_e = 9.1093837015e-28      # g
    c = 2.99792458e10           # cm / s
    pc = 3.0856775814913673e18  # cm
    k = e * e / (2.0 * math.pi * m_e * c)      # cm^3 s^-2 ... per (cm^-3 cm) -> s * Hz^2 * cm^2
    k_astro = k * pc / 1e12                    # DM in pc cm^-3, f in MHz
    assert k_astro == pytest.approx(oracle.K_DM, rel=2e-4)


def test_delay_matches_exact_rational_evaluation():
    """The float64 delay equals floor(k DM (1/f^2 - 1/fref^2) / tsamp + 1/2)
    evaluated exactly on the same inputs, except within 1e-9 of a tie."""
    rng = np.random.default_rng(11)
    fref = 1712.0
    checked = 0
    for _ in range(3000):
        dm = float(rng.uniform(0, 3000))
        f = float(rng.uniform(300, fref))
        ts = float(rng.choice([64e-6, 153.12e-6, 306.24e-6, 1e-3]))
        x = Fraction(oracle.K_DM) * Fraction(dm) * (1 / Fraction(f) ** 2 - 1 / Fraction(fref) ** 2) / Fraction(ts)
        exact = math.floor(x + Fraction(1, 2))
        frac = x - math.floor(x)
        if abs(frac - Fraction(1, 2)) < Fraction(1, 10 ** 9):
            continue
        assert int(oracle.delay_samples(dm, f, fref, ts)) == exact
        checked += 1
    assert checked > 2900


def test_delay_special_values():
    f = synth.band_centres(1712, 856, 64)
    fref = f.max()
    assert np.all(oracle.delay_samples(0.0, f, fref, 1e-4) == 0)
    assert np.all(oracle.delay_samples(np.arange(10) * 100.0, fref, fref, 1e-4) == 0)
    d = oracle.delay_samples(500.0, f, fref, 1e-4)
    assert np.all(np.diff(d) >= 0)          # lower frequency (later channel) arrives later
    assert d[-1] > 0
    # Half-up rounding: a float64 delay of exactly 2.5 samples rounds to 3, not
    # to the even 2.  f = 1024, fref = 2048 make 1/f^2 - 1/fref^2 exact, and this
    # tsamp makes the quotient exactly 2.5 in float64.
    tau = (oracle.K_DM * 0.5) * (1.0 / (1024.0 * 1024.0) - 1.0 / (2048.0 * 2048.0))
    ts = tau / 2.5
    assert tau / ts == 2.5
    assert int(oracle.delay_samples(0.5, 1024.0, 2048.0, ts)) == 3
    assert int(oracle.delay_samples(0.5, 1024.0, 2048.0, tau / 2.25)) == 2
    assert int(oracle.delay_samples(0.5, 1024.0, 2048.0, tau / 2.75)) == 3


# ---------------------------------------------------------------------------
# Dedispersion: brute force, and the sub-band method's reductions to it
# ---------------------------------------------------------------------------

def _python_brute(x, freqs, tsamp, dms, nt):
    fref = max(freqs)
    out = []
    for dm in dms:
        row = []
        for t in range(nt):
            acc = 0
            for ch, f in enumerate(freqs):
                acc += int(x[ch][t + int(oracle.delay_samples(dm, f, fref, tsamp))])
            row.append(acc)
        out.append(row)
    return np.array(out, dtype=np.int64)


def test_channel_rows_by_element_loops():
    # The transpose step (Fig. "dedispersion_flow"): element by element on a
    # small block with a channel pitch wider than nchan.
    rng = np.random.default_rng(9)
    x_tf = rng.integers(0, 256, size=(13, 7), dtype=np.uint8)
    got = oracle.channel_rows(x_tf, 5)
    assert got.shape == (5, 13)
    for ch in range(5):
        for t in range(13):
            assert got[ch][t] == x_tf[t][ch]
    with pytest.raises(ValueError):
        oracle.channel_rows(x_tf, 8)


def test_time_major_block_dedisperses_as_its_channel_rows():
    # Recording order does not change the dedispersed series: brute force on
    # the time-major block's channel rows equals brute force on the original.
    freqs = list(synth.band_centres(1400, 1000, 6))
    dms = [0.0, 9.0, 30.0]
    tsamp = 5e-4
    need = 30 + int(oracle.delay_samples(max(dms), min(freqs), max(freqs), tsamp))
    x = synth.uniform_u8(6, need, 6)
    x_tf = np.zeros((need, 16), dtype=np.uint8)
    x_tf[:, :6] = x.T
    y = oracle.dedisperse_brute(oracle.channel_rows(x_tf, 6), freqs, tsamp, dms, 30)
    assert np.array_equal(y, _python_brute(x, freqs, tsamp, dms, 30))


def test_downsample_by_element_loops_and_special_cases():
    rng = np.random.default_rng(12)
    x = rng.integers(0, 256, size=(3, 37), dtype=np.uint8)
    for k in (1, 2, 4, 8):
        got = oracle.downsample(x, k)
        n = 37 // k
        assert got.shape == (3, n)
        for c in range(3):
            for t in range(n):
                s = sum(int(x[c][k * t + i]) for i in range(k))
                # nearest integer to s / k, halves up (exact rational comparison)
                want = math.floor(Fraction(s, k) + Fraction(1, 2))
                assert got[c][t] == want
    assert np.array_equal(oracle.downsample(x, 1), x)                 # k = 1 is the identity
    const = np.full((2, 64), 77, dtype=np.uint8)
    assert np.all(oracle.downsample(const, 8) == 77)                  # constant in, constant out
    ramp = np.tile(np.arange(64, dtype=np.uint8), (1, 1))
    # mean of 2t .. 2t+1 is 2t + 1/2, which rounds up to 2t + 1
    assert np.array_equal(oracle.downsample(ramp, 2)[0], 2 * np.arange(32) + 1)
    with pytest.raises(ValueError):
        oracle.downsample(x, 4, nt_out=10)


def test_downsampled_range_recovers_high_dm_pulse():
    # A dispersed pulse at high DM, downsampled by 4, is found by a plan at 4x
    # the sampling time near its DM: the trial at the true DM collects the
    # whole pulse, and it beats trials far from it.
    nchan, tsamp, k = 64, 2.5e-4, 4
    freqs = synth.band_centres(1500.0, 1100.0, nchan)
    dm_true = 400.0
    fref = max(freqs)
    d = oracle.delay_samples(dm_true, np.asarray(freqs), fref, tsamp).astype(np.int64)
    reach = int(oracle.delay_samples(500.0, min(freqs), fref, tsamp))
    n = k * 1024 + reach + 64
    x = np.full((nchan, n), 100, dtype=np.uint8)
    for ch in range(nchan):
        x[ch, 1000 + d[ch]:1000 + d[ch] + 8] = 140                     # 8 samples wide at full rate
    xd = oracle.downsample(x, k)
    dms = np.linspace(300.0, 500.0, 41)
    y = oracle.dedisperse_brute(xd, freqs, tsamp * k, dms, 1024)
    best = int(np.argmax(y.max(axis=1)))
    assert abs(dms[best] - dm_true) <= 10.0
    assert y[best].max() >= y[0].max() + nchan * 10


def test_brute_force_matches_triple_loop():
    freqs = list(synth.band_centres(1400, 1000, 6))
    dms = [0.0, 3.0, 17.5, 40.0, 41.0]
    tsamp = 5e-4
    fref = max(freqs)
    need = 20 + int(oracle.delay_samples(max(dms), min(freqs), fref, tsamp))
    x = synth.uniform_u8(6, need, 5)
    y = oracle.dedisperse_brute(x, freqs, tsamp, dms, 20)
    assert np.array_equal(y, _python_brute(x, freqs, tsamp, dms, 20))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_one_trial_per_group_is_brute_force(seed):
    plan = _rand_plan(seed, g=1)
    nt = 97
    x = synth.uniform_u8(plan.nchan, nt + plan.overlap, seed)
    ys = oracle.dedisperse_subband(x, plan, nt)
    yb = oracle.dedisperse_brute(x, plan.freqs, plan.tsamp, plan.dms, nt)
    assert np.array_equal(ys, yb)


@pytest.mark.parametrize("seed", [4, 5])
def test_one_channel_per_subband_is_brute_force(seed):
    plan = _rand_plan(seed, nchan=24, nsub=24)
    assert plan.g == plan.ndm
    nt = 64
    x = synth.uniform_u8(plan.nchan, nt + plan.overlap, seed)
    assert np.array_equal(oracle.dedisperse_subband(x, plan, nt),
                          oracle.dedisperse_brute(x, plan.freqs, plan.tsamp, plan.dms, nt))


@pytest.mark.parametrize("seed", [6, 7, 8])
def test_group_representatives_are_brute_force(seed):
    plan = _rand_plan(seed, nchan=64, nsub=8, ndm=40, dm_max=900.0)
    assert 1 < plan.g < plan.ndm
    nt = 80
    x = synth.uniform_u8(plan.nchan, nt + plan.overlap, seed)
    ys = oracle.dedisperse_subband(x, plan, nt)
    yb = oracle.dedisperse_brute(x, plan.freqs, plan.tsamp, plan.dms, nt)
    reps = np.arange(0, plan.ndm, plan.g)
    assert np.array_equal(ys[reps], yb[reps])
    assert not np.array_equal(ys, yb)   # the approximation is real elsewhere


def test_zero_dm_is_channel_sum():
    plan = _rand_plan(9, nchan=48, nsub=6)
    nt = 50
    x = synth.uniform_u8(plan.nchan, nt + plan.overlap, 9)
    ys = oracle.dedisperse_subband(x, plan, nt)
    assert plan.dms[0] == 0.0
    assert np.array_equal(ys[0], x[:, :nt].astype(np.int64).sum(axis=0))


@pytest.mark.parametrize("seed", [10, 11])
def test_two_stages_equal_effective_offset_sum(seed):
    plan = _rand_plan(seed, nchan=96, nsub=12, ndm=57, dm_max=1200.0)
    nt = 123
    x = synth.uniform_u8(plan.nchan, nt + plan.overlap, seed)
    assert np.array_equal(oracle.dedisperse_subband(x, plan, nt),
                          oracle.dedisperse_offsets(x, plan.offsets, nt))


def test_constant_input_gives_nchan_times_value():
    plan = _rand_plan(12)
    nt = 40
    for v in (0, 1, 128, 255):
        x = np.full((plan.nchan, nt + plan.overlap), v, dtype=np.uint8)
        assert np.all(oracle.dedisperse_subband(x, plan, nt) == plan.nchan * v)


def test_linear_in_input():
    plan = _rand_plan(13)
    nt = 33
    a = synth.uniform_u8(plan.nchan, nt + plan.overlap, 1).astype(np.int64)
    b = synth.uniform_u8(plan.nchan, nt + plan.overlap, 2).astype(np.int64)
    ya = oracle.dedisperse_subband(a, plan, nt)
    yb = oracle.dedisperse_subband(b, plan, nt)
    assert np.array_equal(oracle.dedisperse_subband(3 * a + b, plan, nt), 3 * ya + yb)


def test_impulse_response():
    """A single 1 at (ch, tau) shows up at t = tau - off(i, ch) in every row."""
    plan = _rand_plan(14, nchan=40, nsub=5, ndm=30, dm_max=600.0)
    nt = 150
    ch = 31
    tau = plan.overlap + 20
    x = np.zeros((plan.nchan, nt + plan.overlap), dtype=np.uint8)
    x[ch, tau] = 1
    y = oracle.dedisperse_subband(x, plan, nt)
    for i in range(plan.ndm):
        t = tau - int(plan.offsets[i, ch])
        expect = np.zeros(nt, dtype=np.int64)
        if 0 <= t < nt:
            expect[t] = 1
        assert np.array_equal(y[i], expect)


def test_block_split_invariance():
    """Dedispersing [0, a) and [a, a + b) of one stream equals [0, a + b)."""
    plan = _rand_plan(15)
    a, b = 37, 58
    x = synth.uniform_u8(plan.nchan, a + b + plan.overlap, 15)
    whole = oracle.dedisperse_subband(x, plan, a + b)
    first = oracle.dedisperse_subband(x[:, :a + plan.overlap], plan, a)
    second = oracle.dedisperse_subband(x[:, a:], plan, b)
    assert np.array_equal(np.concatenate([first, second], axis=1), whole)


def test_input_length_is_exactly_output_plus_overlap():
    plan = _rand_plan(16)
    nt = 10
    x = synth.uniform_u8(plan.nchan, nt + plan.overlap, 16)
    oracle.dedisperse_subband(x, plan, nt)
    with pytest.raises(ValueError):
        oracle.dedisperse_subband(x[:, :-1], plan, nt)
    assert plan.overlap >= plan.offsets.max()
    assert plan.overlap >= int(oracle.delay_samples(plan.dms[-1], plan.freqs.min(), plan.fref, plan.tsamp))


@pytest.mark.parametrize("name", ["plain-256", "paper-4096", "octave-8192"])
def test_group_rule_bounds_subband_smearing(name):
    """The coarse grid's promise: the sub-band method's per-channel offset
    differs from the brute-force delay by at most half the full-band delay
    change of one fine DM step, plus the rounding of the four delays."""
    wl = synth.workload(name)
    plan = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    step = float(np.max(np.diff(wl.dms)))
    a_full = 1.0 / plan.freqs.min() ** 2 - 1.0 / plan.fref ** 2
    half_step_delay = 0.5 * oracle.K_DM * step * a_full / plan.tsamp
    rows = np.linspace(0, plan.ndm - 1, 97).astype(int)
    brute = oracle.delay_samples(plan.dms[rows][:, None], plan.freqs[None, :], plan.fref, plan.tsamp)
    err = np.abs(plan.offsets[rows] - brute)
    assert err.max() <= half_step_delay + 2.0
    # and the rule is not trivially loose: one more trial per group breaks it
    plan2 = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub, g=2 * plan.g + 2)
    brute2 = oracle.delay_samples(plan2.dms[rows][:, None], plan2.freqs[None, :], plan2.fref, plan2.tsamp)
    assert np.abs(plan2.offsets[rows] - brute2).max() > half_step_delay + 2.0


def test_plain256_plan_matches_hand_values():
    """256 channels, 16 sub-bands: the coarse groups, overlap and the brute
    reach checked by hand from the delay formula."""
    wl = synth.workload("plain-256")
    plan = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    fmin, fref = wl.freqs.min(), wl.freqs.max()
    reach = oracle.K_DM * 508.0 * (1 / fmin ** 2 - 1 / fref ** 2) / wl.tsamp
    assert plan.overlap == math.floor(reach + 0.5)
    assert plan.g == 4 and plan.ngroups == 32


# ---------------------------------------------------------------------------
# Matched filter (Sec. 2.4)
# ---------------------------------------------------------------------------

def test_window_sums_from_running_sum_equal_direct_sums():
    y = synth.uniform_i32(1, 300, 3, -1000, 1000)[0]
    p = oracle.ref._prefix(y)
    for w in (1, 2, 3, 7, 64, 300):
        S = oracle.ref._window_sums(p, w)
        direct = np.array([int(np.sum(y[t:t + w].astype(np.int64))) for t in range(300 - w + 1)])
        assert np.array_equal(S, direct)


def test_stats_are_population_moments():
    y = synth.uniform_i32(1, 5000, 4, 0, 2_000_000)[0]
    st = oracle.dm_stats(y)
    assert st.sum_y == int(np.sum(y.astype(np.int64)))
    assert st.var == pytest.approx(np.var(y.astype(np.float64)), rel=1e-11)
    assert st.sigma == pytest.approx(np.std(y.astype(np.float64)), rel=1e-11)


def test_snr_is_mean_removed_sum_over_sigma_root_w():
    y = synth.uniform_i32(1, 777, 5, 0, 5000)[0]
    st = oracle.dm_stats(y)
    mean = st.sum_y / 777
    for S, w in ((123456, 32), (1, 1), (4000 * 8, 8), (0, 4)):
        want = (S - w * mean) / (st.sigma * math.sqrt(w))
        assert oracle.snr_from_sum(S, w, 777, st.sum_y, st.inv_d) == pytest.approx(want, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("W", [3, 8, 16, 40])
def test_width_mismatch_loss_closed_form(W):
    """Sec. 2.4, Eq. 8: S/N / S/N_opt = sqrt((W + dW) / W) for dW <= 0 and
    sqrt(W / (W + dW)) for dW > 0, on a noise-free boxcar pulse."""
    T = 400
    y = np.zeros(T)
    y[150:150 + W] = 1.0
    widths = list(range(1, 81))
    snr = oracle.boxcar_snr_fixed(y, widths, 0.0, 1.0)
    opt = math.sqrt(W)
    for w, s in zip(widths, snr):
        dW = w - W
        want = math.sqrt((W + dW) / W) if dW <= 0 else math.sqrt(W / (W + dW))
        assert s / opt == pytest.approx(want, abs=1e-12)


def test_false_alarm_rate_matches_erfc():
    """Sec. 2.4, Eq. 6: on white Gaussian noise the fraction of windows with
    S/N >= gamma is erfc(gamma / sqrt 2) / 2, for every width."""
    rng = np.random.Generator(np.random.PCG64(77))
    T = 1 << 20
    y = np.rint(1000.0 * rng.standard_normal(T)).astype(np.int64)
    for gamma in (2.0, 3.0):
        p = 0.5 * math.erfc(gamma / math.sqrt(2.0))
        for w in (1, 4, 32):
            snr = oracle.boxcar_snr_series(y, w)
            frac = float(np.mean(snr >= gamma))
            se = math.sqrt(p * (1 - p) / (T / w))
            assert abs(frac - p) < 5 * se, (gamma, w, frac, p)


def _brute_peak(y, widths):
    T = len(y)
    st = oracle.dm_stats(y)
    if not st.var > 0:
        return (0.0, widths[0], 0)
    best = None
    for w in sorted(widths):
        if w > T:
            continue
        bS, bt = None, None
        for t in range(T - w + 1):
            S = int(sum(int(v) for v in y[t:t + w]))
            if bS is None or S > bS:
                bS, bt = S, t
        snr = oracle.snr_from_sum(bS, w, T, st.sum_y, st.inv_d)
        if best is None or snr > best[0]:
            best = (snr, w, bt)
    return best if best is not None else (0.0, widths[0], 0)


@pytest.mark.parametrize("seed", range(6))
def test_peak_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    T = int(rng.integers(5, 90))
    y = rng.integers(0, 6, size=T)          # small alphabet: many exact ties
    widths = [1, 2, 4, 8, 16, 32, 64]
    assert oracle.boxcar_peak(y, widths) == _brute_peak(y, widths)


@pytest.mark.parametrize("y,want", [
    ([3, 2, 3, 2, 2, 1, 3, 0, 2], (1, 0)),
    ([3, 1, 3, 2, 3, 2, 0], (1, 0)),
    ([1, 3, 2, 3, 0, 0], (1, 1)),
    ([0, 0, 2, 1, 1, 2], (1, 2)),
])
def test_peak_equal_snr_across_widths_goes_to_smaller_width(y, want):
    """Series where widths 1 and 4 reach bit-identical S/N: the smaller wins."""
    y = np.array(y)
    st = oracle.dm_stats(y)
    T = len(y)
    p = oracle.ref._prefix(y)
    s1 = oracle.ref._window_sums(p, 1).max()
    s4 = oracle.ref._window_sums(p, 4).max()
    assert oracle.snr_from_sum(int(s1), 1, T, st.sum_y, st.inv_d) == \
        oracle.snr_from_sum(int(s4), 4, T, st.sum_y, st.inv_d)
    snr, w, t = oracle.boxcar_peak(y, [1, 2, 4])
    assert (w, t) == want


def test_peak_degenerate_cases():
    assert oracle.boxcar_peak(np.full(50, 7), [2, 4]) == (0.0, 2, 0)
    assert oracle.boxcar_peak(np.arange(3), [4, 8]) == (0.0, 4, 0)
    snr, w, t = oracle.boxcar_peak(np.array([0, 0, 5, 0]), [1, 2, 8])
    assert (w, t) == (1, 2) and snr > 0


@pytest.mark.parametrize("seed", range(4))
def test_candidates_match_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    Y = rng.integers(0, 10, size=(5, 60))
    Y[2, 30:34] += 25
    widths = [1, 2, 4, 8]
    gamma = 2.5
    want = []
    for d in range(5):
        st = oracle.dm_stats(Y[d])
        if not st.var > 0:
            continue
        for t in range(60):
            best = None
            for w in widths:
                if t + w > 60:
                    continue
                S = int(Y[d, t:t + w].sum())
                s = oracle.snr_from_sum(S, w, 60, st.sum_y, st.inv_d)
                if best is None or s > best[1]:
                    best = (w, s)
            if best is not None and best[1] >= gamma:
                want.append((d, t, best[0], best[1]))
    assert oracle.boxcar_candidates(Y, widths, gamma) == want


# ---------------------------------------------------------------------------
# Recovery of injected pulses and the spectral-index loss (Sec. 4.1)
# ---------------------------------------------------------------------------

def _plain256_block():
    wl = synth.workload("plain-256")
    plan = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    _, dm, t0, w, amp = wl.pulses[0]
    start = t0 + oracle.delay_samples(dm, wl.freqs, plan.fref, wl.tsamp)
    x = synth.normal_u8(plan.nchan, wl.nt + plan.overlap, wl.seed, pulses=[(start, w, amp)])
    return wl, plan, x


def test_injected_pulse_recovered_at_its_dm():
    wl, plan, x = _plain256_block()
    yb = oracle.dedisperse_brute(x, plan.freqs, plan.tsamp, plan.dms, wl.nt)
    peaks_b = oracle.boxcar_peaks(yb, wl.widths)
    ib = int(np.argmax(peaks_b[0]))
    assert ib == 50 and plan.dms[ib] == 200.0
    assert peaks_b[2][ib] == 4000 and peaks_b[1][ib] == 4
    ys = oracle.dedisperse_subband(x, plan, wl.nt)
    peaks_s = oracle.boxcar_peaks(ys, wl.widths)
    i_s = int(np.argmax(peaks_s[0]))
    assert i_s == 50
    assert peaks_s[0][i_s] >= 0.5 * peaks_b[0][ib]
    # the zero-variance rule never fires on noise
    assert np.all(peaks_s[0] != 0.0)


def _spectral_closed_form(alpha, eta):
    a = -alpha + 1.0
    b = -2.0 * alpha + 1.0
    return ((eta ** a - 1.0) / a) / math.sqrt((eta - 1.0) * (eta ** b - 1.0) / b)


def test_spectral_index_loss_matches_paper_value():
    v = _paper()["spectral_index_loss_eta2_index2"]
    loss = 1.0 - _spectral_closed_form(-2.0, 2.0)
    assert abs(loss - v["value"]) < v["abs_tolerance"]


def test_spectral_index_dedispersed_pulse_matches_discrete_closed_form():
    """A noise-free pulse with per-channel amplitude a_j, dedispersed at its
    DM, sums to w * sum(a_j); the equal-weight S/N over the optimally weighted
    one is sum(a) / sqrt(N_f sum(a^2)), which approaches the continuum form of
    Sec. 4.1 for many channels."""
    freqs = synth.band_centres(1088.0, 544.0, 256)
    tsamp = 153.12e-6
    dms = np.array([0.0, 250.0, 500.0])
    plan = oracle.make_plan(freqs, tsamp, dms, 16, g=1)
    amps = synth.spectral_amplitudes(freqs, 816.0, -1.5, 3.0)
    nt, w, t0 = 256, 8, 100
    x = np.zeros((256, nt + plan.overlap))
    start = t0 + oracle.delay_samples(500.0, freqs, plan.fref, tsamp)
    for ch in range(256):
        x[ch, start[ch]:start[ch] + w] = amps[ch]
    y = oracle.dedisperse_subband(x, plan, nt)
    assert y[2, t0:t0 + w] == pytest.approx(np.full(w, amps.sum()), rel=1e-12)
    snr_eq = oracle.boxcar_snr_fixed(y[2], [w], 0.0, math.sqrt(256.0))[0]
    snr_opt = w * np.sum(amps ** 2) / (math.sqrt(w) * math.sqrt(np.sum(amps ** 2)))
    ratio = snr_eq / snr_opt
    assert ratio == pytest.approx(amps.sum() / math.sqrt(256 * np.sum(amps ** 2)), rel=1e-12)
    # discrete-channel efficiency vs the continuum closed form (eta = 2)
    f8 = synth.band_centres(1088.0, 544.0, 8192)
    a8 = (f8 / 816.0) ** -1.5
    discrete = a8.sum() / math.sqrt(8192 * np.sum(a8 ** 2))
    assert discrete == pytest.approx(_spectral_closed_form(1.5, 2.0), abs=2e-9)


# ---------------------------------------------------------------------------
# Clustering of the DM-time plane (Sec. 2.5)
# ---------------------------------------------------------------------------

def _plane_points(rng, n_blobs, per_blob, n_noise, ndm, nt, spread):
    pts = set()
    for _ in range(n_blobs):
        d0, t0 = int(rng.integers(5, ndm - 5)), int(rng.integers(50, nt - 50))
        for _ in range(per_blob):
            pts.add((int(np.clip(d0 + rng.integers(-spread, spread + 1), 0, ndm - 1)),
                     int(t0 + rng.integers(-4 * spread, 4 * spread + 1))))
    for _ in range(n_noise):
        pts.add((int(rng.integers(0, ndm)), int(rng.integers(0, nt))))
    return [(d, t, 1, float(rng.uniform(6.0, 20.0))) for d, t in sorted(pts)]


@pytest.mark.parametrize("seed,radius,min_pts", [(1, 4.0, 2), (2, 8.0, 3), (3, 6.5, 0), (4, 16.0, 5)])
def test_dbscan_core_partition_matches_scikit_learn(seed, radius, min_pts):
    # The paper's definitions against an independent DBSCAN: scikit-learn's
    # core points (min_samples counts the point itself, so k + 2 for "more than
    # k others") and its partition of them must agree exactly; its border
    # assignment is order-dependent, so border points are checked for validity.
    from sklearn.cluster import DBSCAN
    rng = np.random.default_rng(seed)
    freqs = synth.band_centres(1712.0, 856.0, 64)
    ndm, nt, tsamp = 200, 2000, 1e-3
    dms = np.arange(ndm) * 0.37 + rng.uniform(0, 0.2)
    pts = _plane_points(rng, 6, 40, 120, ndm, nt, 3)
    srt, lab, reps, ncl = oracle.dbscan_plane(pts, dms, freqs, tsamp, radius, min_pts)
    xs = oracle.delay_axis(dms, freqs, tsamp)
    X = np.array([[xs[d], t] for d, t, _, _ in srt], dtype=np.float64)
    sk = DBSCAN(eps=radius, min_samples=min_pts + 2).fit(X)
    core = np.zeros(len(srt), dtype=bool)
    core[sk.core_sample_indices_] = True
    # our core points are exactly those with a cluster of their own making
    d2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(axis=2)
    ours_core = ((d2 <= radius * radius).sum(axis=1) - 1) > min_pts
    assert np.array_equal(core, ours_core)
    # same partition of the core points
    pairs_sk = {(int(a), int(b)) for a in np.nonzero(core)[0] for b in np.nonzero(core)[0]
                if sk.labels_[a] == sk.labels_[b]}
    pairs_us = {(int(a), int(b)) for a in np.nonzero(core)[0] for b in np.nonzero(core)[0] if lab[a] == lab[b]}
    assert pairs_sk == pairs_us
    assert ncl == len(set(sk.labels_[core]))
    # noise agrees; every border point sits within r of a core point of its cluster
    assert np.array_equal(lab < 0, sk.labels_ < 0)
    for i in np.nonzero(~core & (lab >= 0))[0]:
        near = np.nonzero(core & (d2[i] <= radius * radius))[0]
        assert any(lab[q] == lab[i] for q in near)
    # representatives: the highest S/N of each cluster
    for c in range(ncl):
        members = np.nonzero(lab == c)[0]
        assert srt[reps[c]][3] == max(srt[i][3] for i in members)


def test_dbscan_hand_cases():
    freqs = [1500.0, 1400.0]
    tsamp = 1e-3
    dms = np.zeros(10)                                  # every DM at delay 0: a 1-D problem in time
    chain = [(0, 10 * i, 1, 7.0 + i) for i in range(6)]  # spaced 10 apart
    far = [(0, 500, 1, 9.0), (0, 505, 1, 8.0)]
    pts = chain + far
    srt, lab, reps, ncl = oracle.dbscan_plane(pts, dms, freqs, tsamp, 10.0, 1)
    # interior chain points have 2 neighbours (> 1): core; the ends are reachable
    assert ncl == 1 and list(lab) == [0] * 6 + [-1, -1]
    assert reps[0] == 5                                 # highest S/N, the last of the chain
    srt, lab, reps, ncl = oracle.dbscan_plane(pts, dms, freqs, tsamp, 10.0, 2)
    assert ncl == 0 and np.all(lab == -1)               # no point has more than 2 neighbours
    srt, lab, reps, ncl = oracle.dbscan_plane(pts, dms, freqs, tsamp, 9.99, 0)
    assert ncl == 1 and list(lab) == [-1] * 6 + [0, 0]  # only the close pair is within 9.99
    srt, lab, reps, ncl = oracle.dbscan_plane([], dms, freqs, tsamp, 5.0, 1)
    assert ncl == 0 and len(lab) == 0


def test_delay_axis_rounds_to_the_plan_delay_of_the_lowest_channel():
    freqs = synth.band_centres(1712.0, 856.0, 256)
    dms = np.array([0.0, 3.5, 100.0, 1234.5])
    x = oracle.delay_axis(dms, freqs, 306.24e-6)
    d = oracle.delay_samples(dms, freqs.min(), freqs.max(), 306.24e-6)
    assert np.array_equal(np.floor(x + 0.5).astype(np.int64), d)


# ---------------------------------------------------------------------------
# Narrow-band RFI: channel statistics and mask (Sec. 2.2)
# ---------------------------------------------------------------------------

def test_power_sums_by_loops():
    rng = np.random.default_rng(31)
    x = rng.integers(0, 256, size=(3, 23), dtype=np.uint8)
    s = oracle.channel_power_sums(x)
    for c in range(3):
        for j in range(4):
            assert s[c][j] == sum(int(v) ** (j + 1) for v in x[c])


def test_moments_match_scipy_and_closed_forms():
    from scipy import stats
    rng = np.random.default_rng(32)
    x = np.concatenate([rng.integers(0, 256, size=(4, 5000)), np.full((1, 5000), 7),
                        np.tile([0, 2], (1, 2500))]).astype(np.uint8)
    mom = oracle.channel_moments(oracle.channel_power_sums(x), 5000)
    for c in range(4):
        g1, b2 = mom[c]
        assert g1 == pytest.approx(stats.skew(x[c].astype(np.float64)), rel=1e-9, abs=1e-12)
        assert b2 == pytest.approx(stats.kurtosis(x[c].astype(np.float64), fisher=False), rel=1e-9)
    assert mom[4] is None                       # constant channel: no variance
    assert mom[5] == (0.0, 1.0)                 # two equal point masses: skew 0, kurtosis 1


def test_skf_mask_removes_planted_rfi_channels():
    # Noise channels plus: an impulsive channel (rare spikes: huge kurtosis),
    # a skewed channel (one-sided bursts), a constant channel.
    x = synth.normal_u8(40, 8000, 33)
    x[5] = 128
    x[5, ::97] = 255
    x[17] = np.clip(x[17].astype(np.int64) + (np.arange(8000) % 50 < 5) * 90, 0, 255).astype(np.uint8)
    x[30] = 128
    mask = oracle.skf_mask(oracle.channel_power_sums(x), 8000, 5.0)
    assert list(np.nonzero(mask == 0)[0]) == [5, 17, 30]


def test_masked_channels_count_as_zero_rows():
    plan = _rand_plan(34)
    x = synth.uniform_u8(32, 400 + plan.overlap, 35)
    mask = np.ones(32, dtype=np.uint8)
    mask[[0, 3, 31]] = 0
    xz = x * mask[:, None]
    y = oracle.dedisperse_subband(xz, plan, 400)
    # one channel's removal subtracts exactly its own delayed row
    y_all = oracle.dedisperse_subband(x, plan, 400)
    y_one = oracle.dedisperse_subband(x * (np.arange(32) != 3)[:, None].astype(np.uint8), plan, 400)
    off = plan.offsets[:, 3]
    for i in range(plan.ndm):
        assert np.array_equal(y_all[i] - y_one[i], x[3, off[i]:off[i] + 400])
    assert y.dtype == np.int64


# ---------------------------------------------------------------------------
# Normalisation (Sec. 2.1) and the float path
# ---------------------------------------------------------------------------

def test_norm_weights_closed_forms():
    """A channel alternating a and b has mean (a+b)/2 and sigma |a-b|/2, so
    unit weighting maps it to exactly -1, +1 and inverse-variance weighting
    to -1/sigma, +1/sigma; a constant channel is dropped (0, 0)."""
    n = 64
    x = np.zeros((3, n), dtype=np.uint8)
    x[0, 0::2], x[0, 1::2] = 100, 132            # mean 116, sigma 16
    x[1, 0::2], x[1, 1::2] = 7, 9                # mean 8, sigma 1
    x[2] = 77                                    # constant
    sums = oracle.channel_power_sums(x)
    mv = oracle.channel_mean_var(sums, n)
    assert mv[0] == (116.0, 256.0) and mv[1] == (8.0, 1.0) and mv[2] == (77.0, 0.0)
    s, o = oracle.norm_weights(sums, n, oracle.WEIGHT_UNIT)
    assert (s[0], o[0], s[1], o[1], s[2], o[2]) == (1 / 16, 116 / 16, 1.0, 8.0, 0.0, 0.0)
    v = oracle.normalise(x, s, o)
    assert np.array_equal(v[0], np.where(x[0] == 132, 1.0, -1.0))
    assert np.array_equal(v[1], np.where(x[1] == 9, 1.0, -1.0))
    assert np.array_equal(v[2], np.zeros(n))
    s, o = oracle.norm_weights(sums, n, oracle.WEIGHT_INVERSE_VAR)
    v = oracle.normalise(x, s, o)
    assert np.array_equal(v[0], np.where(x[0] == 132, 1.0 / 16, -1.0 / 16))
    assert np.array_equal(v[1], np.where(x[1] == 9, 1.0, -1.0))


@pytest.mark.parametrize("seed", [1, 2])
def test_normalised_channels_have_zero_mean_and_unit_variance(seed):
    rng = np.random.default_rng(seed)
    nchan, n = 24, 5000
    sig = rng.uniform(2.0, 40.0, size=nchan)
    mu = rng.uniform(60.0, 190.0, size=nchan)
    x = np.clip(np.rint(mu[:, None] + sig[:, None] * rng.standard_normal((nchan, n))), 0, 255).astype(np.uint8)
    sums = oracle.channel_power_sums(x)
    for (m, v), row in zip(oracle.channel_mean_var(sums, n), x):
        assert math.isclose(m, float(np.mean(row, dtype=np.float64)), rel_tol=1e-13)
        assert math.isclose(v, float(np.var(row, dtype=np.float64)), rel_tol=1e-12)
    s, o = oracle.norm_weights(sums, n, oracle.WEIGHT_UNIT)
    y = oracle.normalise(x, s, o)
    assert np.all(np.abs(y.mean(axis=1)) < 1e-5)             # float32 weights: ~1e-7 relative
    assert np.all(np.abs(y.var(axis=1) - 1.0) < 1e-5)
    s, o = oracle.norm_weights(sums, n, oracle.WEIGHT_INVERSE_VAR)
    y = oracle.normalise(x, s, o)
    var = np.array([v for _, v in oracle.channel_mean_var(sums, n)])
    assert np.all(np.abs(y.var(axis=1) * var - 1.0) < 1e-5)  # variance 1 / sigma^2


def test_normalised_dedispersion_is_affine_in_the_integer_one():
    """With one scale s and offset o for every channel, the two stages of the
    normalised block are exactly s * Y - nchan * o, Y the (pinned) integer
    two-stage result (s = 1/16 and o = 8 keep every float64 sum exact)."""
    freqs = synth.band_centres(1712.0, 856.0, 64)
    dms = np.linspace(0.0, 300.0, 40)
    plan = oracle.make_plan(freqs, 306.24e-6, dms, 8)
    nt = 700
    x = synth.uniform_u8(64, nt + plan.overlap, 5)
    s = np.full(64, 1.0 / 16)
    o = np.full(64, 8.0)
    got = oracle.dedisperse_subband_norm(x, plan, nt, s, o)
    want = oracle.dedisperse_subband(x, plan, nt).astype(np.float64) / 16.0 - 64 * 8.0
    assert np.array_equal(got, want)


def test_inverse_variance_weights_give_the_matched_snr():
    """Half the channels noisy (sigma 32), half quiet (sigma 8), the same
    raw amplitude A in every channel for 40 pulses of width w (DM 0).  After
    normalisation and the channel sum, a pulse's S/N (against the noise of
    the pulse-free samples) is A sqrt(w) sum(1/sigma) / sqrt(N) with unit
    weights and A sqrt(w) sqrt(sum 1/sigma^2) with inverse-variance weights,
    the largest any channel weighting reaches.  The mean over the 40 pulses
    is within 3% of each closed form (its noise is about 0.8%)."""
    rng = np.random.default_rng(11)
    nchan, n, w, A, npulse = 32, 40000, 8, 16.0, 40
    sig = np.where(np.arange(nchan) < nchan // 2, 32.0, 8.0)
    z = 128.0 + sig[:, None] * rng.standard_normal((nchan, n))
    starts = 500 + 900 * np.arange(npulse)
    for t0 in starts:
        z[:, t0:t0 + w] += A
    x = np.clip(np.rint(z), 0, 255).astype(np.uint8)
    sums = oracle.channel_power_sums(x)
    quiet = np.ones(n, dtype=bool)
    for t0 in starts:
        quiet[t0 - w:t0 + 2 * w] = False
    got = {}
    for mode in (oracle.WEIGHT_UNIT, oracle.WEIGHT_INVERSE_VAR):
        s, o = oracle.norm_weights(sums, n, mode)
        y = oracle.normalise(x, s, o).sum(axis=0)
        mu, sd = y[quiet].mean(), y[quiet].std()
        got[mode] = np.mean([(y[t0:t0 + w].sum() - w * mu) / (sd * math.sqrt(w)) for t0 in starts])
    unit = A * math.sqrt(w) * np.sum(1.0 / sig) / math.sqrt(nchan)
    ivar = A * math.sqrt(w) * math.sqrt(np.sum(1.0 / sig ** 2))
    assert abs(got[oracle.WEIGHT_UNIT] / unit - 1.0) < 0.03
    assert abs(got[oracle.WEIGHT_INVERSE_VAR] / ivar - 1.0) < 0.03
    assert got[oracle.WEIGHT_INVERSE_VAR] > got[oracle.WEIGHT_UNIT]


@pytest.mark.parametrize("seed", [3, 4])
def test_float_boxcar_equals_integer_boxcar_on_integer_series(seed):
    """On integer-valued series the float matched filter and the (pinned)
    integer one agree: the same width and start, S/N to 1e-9 (they form the
    variance by different exact-ish routes), and the same candidates."""
    rng = np.random.default_rng(seed)
    Y = rng.integers(0, 300, size=(6, 3000)).astype(np.int32)
    Y[1, 1000:1016] += 90
    Y[4, 2990:] += 200
    widths = [1, 2, 4, 8, 16, 32]
    fs, fw, ft = oracle.boxcar_peaks_float(Y.astype(np.float64), widths)
    is_, iw, it = oracle.boxcar_peaks(Y, widths)
    assert np.array_equal(fw, iw) and np.array_equal(ft, it)
    assert np.allclose(fs, is_, rtol=1e-9, atol=0)
    gamma = 3.0
    fc = oracle.boxcar_candidates_float(Y.astype(np.float64), widths, gamma)
    ic = oracle.boxcar_candidates(Y, widths, gamma)
    assert all(abs(c[3] - gamma) > 1e-6 for c in ic)
    assert [c[:3] for c in fc] == [c[:3] for c in ic]
    assert np.allclose([c[3] for c in fc], [c[3] for c in ic], rtol=1e-9, atol=0)
