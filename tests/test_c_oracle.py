"""The C oracle (OpenMP) against the NumPy oracle and brute force: two
independent restatements of the same definitions must agree exactly."""

import numpy as np
import pytest

import oracle
import synth
from oracle import c_oracle as co


def _shapes():
    return [
        (64, 8, 40, 300.0, 1712.0, 856.0, 306.24e-6, 3000),
        (128, 16, 61, 700.0, 1712.0, 856.0, 306.24e-6, 2049),
        (96, 12, 33, 1500.0, 1088.0, 544.0, 153.12e-6, 1500),
        (48, 48, 20, 400.0, 1500.0, 1100.0, 5e-4, 777),
        (60, 1, 25, 200.0, 1500.0, 1100.0, 1e-3, 999),
    ]


@pytest.mark.parametrize("name", ["plain-256", "paper-4096", "served-4096", "octave-8192"])
def test_plan_tables_equal_numpy_oracle(name):
    wl = synth.workload(name)
    ref = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    assert co.group_size_rule(wl.freqs, wl.nsub, len(wl.dms)) == ref.g
    cc, cs, fs, o = co.plan_tables(wl.freqs, wl.tsamp, wl.dms, wl.nsub, ref.g)
    assert np.array_equal(cc, ref.d_coarse_chan)
    assert np.array_equal(cs, ref.d_coarse_sub)
    assert np.array_equal(fs, ref.d_fine_sub)
    assert o == ref.overlap


@pytest.mark.parametrize("shape", _shapes())
@pytest.mark.parametrize("g_mode", ["rule", "one", "all"])
def test_subband_equals_numpy_oracle(shape, g_mode):
    nchan, nsub, ndm, dmmax, ft, fb, ts, nt = shape
    freqs = synth.band_centres(ft, fb, nchan)
    dms = np.linspace(0.0, dmmax, ndm)
    g = {"rule": None, "one": 1, "all": ndm}[g_mode]
    ref = oracle.make_plan(freqs, ts, dms, nsub, g=g)
    x = synth.uniform_u8(nchan, nt + ref.overlap, 11 + nchan)
    want = oracle.dedisperse_subband(x, ref, nt)
    got = co.dedisperse_subband(x, freqs, ts, dms, nsub, ref.g, nt, threads=3)
    assert np.array_equal(got, want)


def test_brute_equals_numpy_oracle_and_threads_agree():
    freqs = synth.band_centres(1712.0, 856.0, 64)
    dms = np.linspace(0.0, 250.0, 30)
    ref = oracle.make_plan(freqs, 306.24e-6, dms, 8)
    x = synth.uniform_u8(64, 2000 + ref.overlap, 5)
    want = oracle.dedisperse_brute(x, freqs, 306.24e-6, dms, 2000)
    assert np.array_equal(co.dedisperse_brute(x, freqs, 306.24e-6, dms, 2000, threads=1), want)
    assert np.array_equal(co.dedisperse_brute(x, freqs, 306.24e-6, dms, 2000, threads=4), want)


def test_boxcar_peaks_and_candidates_equal_numpy_oracle():
    rng = np.random.Generator(np.random.PCG64(9))
    T = 3000
    Y = rng.integers(1000, 1200, size=(12, T)).astype(np.int32)
    Y[3, 1000:1008] += 400                 # a pulse
    Y[4, :] = 777                          # zero variance
    Y[5, 2990:] += 300                     # a pulse at the block end
    widths = [1, 2, 4, 8, 16, 32, 4096]    # the last is longer than the block
    ws, ww, wt = oracle.boxcar_peaks(Y, widths)
    cs, cw, ct = co.boxcar_peaks(Y, widths, threads=4)
    assert np.array_equal(cs, ws) and np.array_equal(cw, ww) and np.array_equal(ct, wt)
    for gamma in (3.0, 4.5):
        assert co.boxcar_candidates(Y, widths, gamma, threads=4) == oracle.boxcar_candidates(Y, widths, gamma)


def test_plain256_end_to_end_matches_numpy_oracle():
    wl = synth.workload("plain-256")
    ref = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    start = 4000 + oracle.delay_samples(200.0, wl.freqs, ref.fref, wl.tsamp)
    x = synth.normal_u8(256, wl.nt + ref.overlap, 1, pulses=[(start, 4, 96.0)])
    y = co.dedisperse_subband(x, wl.freqs, wl.tsamp, wl.dms, wl.nsub, ref.g, wl.nt)
    want = oracle.dedisperse_subband(x, ref, wl.nt)
    assert np.array_equal(y, want)
    assert co.boxcar_candidates(y, wl.widths, 6.0) == oracle.boxcar_candidates(want, wl.widths, 6.0)
