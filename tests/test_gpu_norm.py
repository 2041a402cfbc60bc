"""The normalised (floating-point) variant through the C ABI: per-channel
weights from the device's exact power sums, dedispersion of the normalised
block in float32 against the oracle's float64 within the stated rounding
bound, and the float matched filter against the oracle on the same float32
series."""

import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2401_13834_amd as tx
from gpu_helpers import as_tuples, device_block, torch_cuda

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _varied_block(nchan, n, seed):
    """Channels of different means and spreads (the case normalisation is for)."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(60.0, 190.0, size=nchan)
    sig = rng.uniform(3.0, 30.0, size=nchan)
    z = mu[:, None] + sig[:, None] * rng.standard_normal((nchan, n))
    x = np.clip(np.rint(z), 0, 255).astype(np.uint8)
    x[nchan // 3] = 100                          # a constant channel: weight 0
    return x


def _weights_gpu(torch, d_in, nchan, n, weighting):
    sums = torch.empty((nchan, 4), dtype=torch.int64, device="cuda")
    tx.tx_channel_power_sums(d_in, nchan, n, sums)
    torch.cuda.synchronize()
    h = sums.cpu().numpy()
    scale, offset = tx.tx_norm_weights(h, n, weighting)
    return h, scale, offset


SHAPES = [  # (nchan, nsub, ndm, nt, f_top, f_bot, tsamp, dm_max)
    (64, 8, 40, 3000, 1712.0, 856.0, 306.24e-6, 300.0),
    (256, 16, 100, 5000, 1712.0, 856.0, 153.12e-6, 500.0),
    (96, 12, 57, 1025, 1500.0, 1100.0, 1e-3, 1200.0),
    (48, 48, 33, 777, 1500.0, 1100.0, 5e-4, 900.0),
    (1024, 64, 60, 2100, 1712.0, 856.0, 153.12e-6, 1000.0),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"s{i}" for i in range(len(SHAPES))])
@pytest.mark.parametrize("weighting", [0, 1])
def test_dedisperse_norm_within_rounding_bound(shape, weighting):
    torch = torch_cuda()
    nchan, nsub, ndm, nt, ft, fb, ts, dmmax = shape
    _say(f"norm shape={shape} weighting={weighting}")
    freqs = synth.band_centres(ft, fb, nchan)
    dms = np.linspace(0.0, dmmax, ndm)
    ref = oracle.make_plan(freqs, ts, dms, nsub)
    plan = tx.tx_plan(freqs, ts, dms, nsub)
    n = nt + ref.overlap
    x = _varied_block(nchan, n, nchan + ndm)
    d_in = device_block(x)
    sums, scale, offset = _weights_gpu(torch, d_in, nchan, n, weighting)
    ws, wo = oracle.norm_weights(sums, n, weighting)
    assert np.array_equal(scale.astype(np.float64), ws) and np.array_equal(offset.astype(np.float64), wo)
    d_s = torch.from_numpy(scale).to("cuda")
    d_o = torch.from_numpy(offset).to("cuda")
    out = torch.full((plan.ndm, nt + 5), -7.0, dtype=torch.float32, device="cuda")
    tx.tx_dedisperse_norm(plan, d_in, nt, d_s, d_o, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    want = oracle.dedisperse_subband_norm(x, ref, nt, ws, wo)
    bound = (ref.m + ref.nsub + 1) * U * oracle.norm_abs_bound(x, ref, nt, ws, wo)
    err = np.abs(got[:, :nt] - want)
    assert np.all(err <= bound), float(np.max(err / np.maximum(bound, 1e-300)))
    assert np.all(got[:, nt:] == -7.0)
    if weighting == 0:
        # normalised noise: every trial's series has mean ~0 and std ~sqrt(channels kept)
        assert abs(float(np.mean(want[0]))) < 0.2 * np.sqrt(nchan)


W7 = [1, 2, 4, 8, 16, 32, 64]


@pytest.mark.parametrize("nt,seed,widths", [(5, 1, W7), (4096, 2, W7), (4097, 3, W7), (10000, 4, W7),
                                            (9000, 5, list(range(1, 33))), (20000, 6, [3, 5, 100, 1000]),
                                            (70001, 7, [1 << k for k in range(10)])])
def test_float_boxcar_matches_oracle_on_the_same_series(nt, seed, widths):
    torch = torch_cuda()
    _say(f"float boxcar nt={nt} widths={len(widths)}")
    rng = np.random.default_rng(seed)
    rows = 12
    Y = rng.standard_normal((rows, nt)).astype(np.float32) * 8.0
    Y[1] = 3.25                                  # zero variance
    Y[3, nt // 2] += 60.0
    Y[4, :min(nt, 40)] += 9.0
    Y[5, -min(nt, 3):] += 30.0
    d = torch.from_numpy(Y).to("cuda")
    snr = torch.empty(rows, dtype=torch.float64, device="cuda")
    wid = torch.empty(rows, dtype=torch.int32, device="cuda")
    tim = torch.empty(rows, dtype=torch.int64, device="cuda")
    cap = 1 << 16
    raw = torch.zeros((cap, 3), dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    gamma = 3.0
    tx.tx_candidates_f32(d, nt, widths, gamma, raw, cnt, peaks=(snr, wid, tim))
    torch.cuda.synchronize()
    Yd = Y.astype(np.float64)
    ws, ww, wt = oracle.boxcar_peaks_float(Yd, widths)
    gs, gw, gt = snr.cpu().numpy(), wid.cpu().numpy(), tim.cpu().numpy()
    assert np.allclose(gs, ws, rtol=1e-9, atol=1e-12)
    for r in range(rows):
        if (gw[r], gt[r]) != (ww[r], wt[r]):     # a near tie: the GPU's pick must be as good
            s = oracle.boxcar_snr_series_float(Yd[r], int(gw[r]))[int(gt[r])]
            assert abs(s - ws[r]) <= 1e-9 * abs(ws[r])
    n = int(cnt.item())
    got = as_tuples(tx.parse_candidates(raw.cpu().numpy(), n))
    want = oracle.boxcar_candidates_float(Yd, widths, gamma)
    gd = {(c[0], c[1]): c for c in got}
    wd = {(c[0], c[1]): c for c in want}
    for k in set(gd) ^ set(wd):                  # only points at the threshold may differ
        c = gd.get(k) or wd.get(k)
        assert abs(c[3] - gamma) < 1e-9 * gamma, c
    for k in set(gd) & set(wd):
        assert abs(gd[k][3] - wd[k][3]) <= 1e-9 * abs(wd[k][3])
    tx.tx_boxcar_snr_f32(d, nt, widths, snr, wid, tim)
    torch.cuda.synchronize()
    assert np.array_equal(snr.cpu().numpy(), gs) and np.array_equal(tim.cpu().numpy(), gt)


def test_normalised_path_recovers_a_pulse_in_uneven_channels():
    """plain-256's pulse (DM 200, width 4) in channels whose noise levels
    differ eightfold: through the power sums, inverse-variance weights, the
    float dedispersion and the float matched filter on the device, the pulse
    is found at its trial and time, and the S/N matches the oracle's on the
    same float32 output."""
    torch = torch_cuda()
    wl = synth.workload("plain-256")
    ref = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    nchan, nt = 256, wl.nt
    n = nt + ref.overlap
    rng = np.random.default_rng(21)
    sig = np.where(np.arange(nchan) % 2 == 0, 4.0, 32.0)
    z = 128.0 + sig[:, None] * rng.standard_normal((nchan, n))
    start = 4000 + oracle.delay_samples(200.0, wl.freqs, ref.fref, wl.tsamp)
    for c in range(nchan):
        z[c, start[c]:start[c] + 4] += 12.0
    x = np.clip(np.rint(z), 0, 255).astype(np.uint8)
    d_in = device_block(x)
    _, scale, offset = _weights_gpu(torch, d_in, nchan, n, tx.TX_WEIGHT_INVERSE_VAR)
    out = torch.empty((plan.ndm, nt), dtype=torch.float32, device="cuda")
    tx.tx_dedisperse_norm(plan, d_in, nt, torch.from_numpy(scale).to("cuda"), torch.from_numpy(offset).to("cuda"),
                          out)
    snr = torch.empty(plan.ndm, dtype=torch.float64, device="cuda")
    wid = torch.empty(plan.ndm, dtype=torch.int32, device="cuda")
    tim = torch.empty(plan.ndm, dtype=torch.int64, device="cuda")
    tx.tx_boxcar_snr_f32(out, nt, wl.widths, snr, wid, tim)
    torch.cuda.synchronize()
    s = snr.cpu().numpy()
    best = int(np.argmax(s))
    assert best == 50 and abs(int(tim[best].item()) - 4000) <= 4
    Y = out.cpu().numpy().astype(np.float64)
    ws, _, _ = oracle.boxcar_peaks_float(Y[best:best + 1], wl.widths)
    assert abs(s[best] - ws[0]) <= 1e-9 * ws[0]


@pytest.mark.parametrize("W", [4, 16, 64])
def test_fixed_sigma_boxcar_width_mismatch_closed_form(W):
    """Sec. 2.4's width mismatch on the GPU path: a noise-free boxcar pulse
    of width W and unit amplitude, searched with width w and a fixed sigma,
    has S/N sqrt(w) for w <= W and W / sqrt(w) for w >= W (relative to its
    matched S/N sqrt(W): sqrt(w/W) and sqrt(W/w)), to 1e-12."""
    torch = torch_cuda()
    nt = 9000
    y = np.zeros((1, nt), dtype=np.float32)
    y[0, 3000:3000 + W] = 1.0
    widths = [1, 2, 4, 8, 16, 32, 64, 128, 256]
    d = torch.from_numpy(y).to("cuda")
    for w in widths:
        snr = torch.empty(1, dtype=torch.float64, device="cuda")
        wid = torch.empty(1, dtype=torch.int32, device="cuda")
        tim = torch.empty(1, dtype=torch.int64, device="cuda")
        tx.tx_boxcar_snr_fixed(d, nt, [w], 0.0, 1.0, snr, wid, tim)
        torch.cuda.synchronize()
        want = np.sqrt(w) if w <= W else W / np.sqrt(w)
        assert abs(float(snr.item()) - want) <= 1e-12 * want
        assert np.isclose(float(snr.item()) / np.sqrt(W), np.sqrt(min(w, W) / max(w, W)), rtol=1e-12)
        assert float(snr.item()) == pytest.approx(oracle.boxcar_snr_fixed(y[0], [w], 0.0, 1.0)[0], rel=1e-12)
    # the matched width wins, at the pulse's start
    snr = torch.empty(1, dtype=torch.float64, device="cuda")
    wid = torch.empty(1, dtype=torch.int32, device="cuda")
    tim = torch.empty(1, dtype=torch.int64, device="cuda")
    tx.tx_boxcar_snr_fixed(d, nt, widths, 0.0, 1.0, snr, wid, tim)
    torch.cuda.synchronize()
    assert int(wid.item()) == W and int(tim.item()) == 3000
    with pytest.raises(tx.TxError):
        tx.tx_boxcar_snr_fixed(d, nt, widths, 0.0, 0.0, snr, wid, tim)


@pytest.mark.parametrize("widths,nt", [(list(range(1, 33)), 600001),
                                       (sorted([1 << k for k in range(11)] + [3, 5, 6, 7, 12, 24, 48, 96, 200]), 1 << 20)])
def test_float_boxcar_long_rows_without_tile_table(widths, nt):
    """Float rows too long for the filter's per-(tile, width) table (tiles of
    4096 starts x width slots x 8 bytes over 16 KB): candidates then come from
    a second scan of every tile."""
    torch = torch_cuda()
    assert -(-nt // 4096) * 32 * 8 > 16 * 1024
    _say(f"float boxcar long rows nt={nt} widths={len(widths)}")
    rng = np.random.default_rng(nt)
    Y = rng.standard_normal((3, nt)).astype(np.float32) * 5.0
    Y[0, nt - 3:] += 40.0
    Y[1, ::40961] += 60.0
    Y[2, 123456:123470] += 25.0
    d = torch.from_numpy(Y).to("cuda")
    rows = Y.shape[0]
    snr = torch.empty(rows, dtype=torch.float64, device="cuda")
    wid = torch.empty(rows, dtype=torch.int32, device="cuda")
    tim = torch.empty(rows, dtype=torch.int64, device="cuda")
    raw = torch.zeros((1 << 16, 3), dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    gamma = 6.0
    tx.tx_candidates_f32(d, nt, widths, gamma, raw, cnt, peaks=(snr, wid, tim))
    torch.cuda.synchronize()
    Yd = Y.astype(np.float64)
    ws, ww, wt = oracle.boxcar_peaks_float(Yd, widths)
    gs, gw, gt = snr.cpu().numpy(), wid.cpu().numpy(), tim.cpu().numpy()
    assert np.allclose(gs, ws, rtol=1e-9, atol=1e-12)
    for r in range(rows):
        if (gw[r], gt[r]) != (ww[r], wt[r]):     # a near tie: the GPU's pick must be as good
            s = oracle.boxcar_snr_series_float(Yd[r], int(gw[r]))[int(gt[r])]
            assert abs(s - ws[r]) <= 1e-9 * abs(ws[r])
    n = int(cnt.item())
    got = {(c[0], c[1]): c for c in as_tuples(tx.parse_candidates(raw.cpu().numpy(), n))}
    want = {(c[0], c[1]): c for c in oracle.boxcar_candidates_float(Yd, widths, gamma)}
    assert len(want) > 0
    for k in set(got) ^ set(want):               # only points at the threshold may differ
        c = got.get(k) or want.get(k)
        assert abs(c[3] - gamma) < 1e-9 * gamma, c
    for k in set(got) & set(want):
        assert abs(got[k][3] - want[k][3]) <= 1e-9 * abs(want[k][3])
