"""Seeded random shapes through the C ABI against the oracle: bands, channel
and sub-band counts, DM grids (uniform and irregular), DMs per group (the
smearing rule or given), block lengths, first- and second-stage tile
variants with their LDS sizes, and boxcar width lists.  Dedispersion outputs
and candidate lists must be bit-exact, S/N equal."""

import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2401_13834_amd as tx
from gpu_helpers import as_tuples, gpu_candidates, gpu_dedisperse, torch_cuda

pytestmark = pytest.mark.gpu

N_SHAPES = 24


def _shape(seed):
    rng = np.random.default_rng(1000 + seed)
    nchan = int(rng.integers(1, 700))
    divs = [d for d in range(1, nchan + 1) if nchan % d == 0 and nchan // d <= 256]
    nsub = int(rng.choice(divs))
    f_top = float(rng.uniform(400.0, 2000.0))
    f_bot = float(rng.uniform(0.3 * f_top, f_top))
    tsamp = float(rng.uniform(5e-5, 1e-3))
    ndm = int(rng.integers(1, 300))
    dm_max = float(rng.uniform(0.0, 1500.0))
    dms = np.sort(rng.uniform(0.0, dm_max, ndm)) if rng.random() < 0.3 else np.linspace(0.0, dm_max, ndm)
    g = 0 if rng.random() < 0.6 else int(rng.integers(1, 41))
    nt = int(rng.integers(1, 6000))
    tiles = (int(rng.integers(-1, len(tx.tx_tile_variants(1)))), int(rng.choice([0, 16384, 27296, 40960, 65536])),
             int(rng.integers(-1, len(tx.tx_tile_variants(2)))), int(rng.choice([0, 8192, 32768, 65536])))
    widths = sorted(set(int(w) for w in rng.integers(1, 300, int(rng.integers(1, 12))) if w <= nt)) or [1]
    gamma = float(rng.uniform(2.5, 4.5))
    return nchan, nsub, f_top, f_bot, tsamp, dms, g, nt, tiles, widths, gamma


def _supported(plan, nt):
    """Whether the plan's tiles can stage their rows for nt outputs (else the
    library answers TX_ENOTSUP: a group of trials spanning a very wide range
    of delays)."""
    try:
        plan.ws_size(nt)
        return True
    except tx.TxError as e:
        assert e.status == tx.TX_ENOTSUP
        return False


@pytest.mark.parametrize("seed", range(N_SHAPES))
def test_random_shape_matches_oracle(seed):
    torch = torch_cuda()
    nchan, nsub, f_top, f_bot, tsamp, dms, g, nt, tiles, widths, gamma = _shape(seed)
    print(f"random shape {seed}: nchan {nchan} nsub {nsub} band {f_top:.1f}-{f_bot:.1f} tsamp {tsamp:.2e} "
          f"ndm {len(dms)} g {g} nt {nt} tiles {tiles} widths {widths} gamma {gamma:.2f}", flush=True)
    sys.stdout.flush()
    freqs = synth.band_centres(f_top, f_bot, nchan)
    ref = oracle.make_plan(freqs, tsamp, dms, nsub, g=None if g == 0 else g)
    plan = tx.tx_plan(freqs, tsamp, dms, nsub, dms_per_group=g)
    assert (plan.g, plan.overlap) == (ref.g, ref.overlap)
    plan.set_tiles(*tiles)
    x = synth.uniform_u8(nchan, nt + ref.overlap, seed)
    if not _supported(plan, nt):
        # a staged row of these tiles does not fit the LDS: refused, not run
        with pytest.raises(tx.TxError) as e:
            gpu_dedisperse(plan, x, nt)
        assert e.value.status == tx.TX_ENOTSUP
        return
    want = oracle.dedisperse_subband(x, ref, nt)
    got = gpu_dedisperse(plan, x, nt)
    assert np.array_equal(got[:, :nt], want)

    d = torch.from_numpy(np.ascontiguousarray(want, dtype=np.int32)).to("cuda")
    n, rec, peaks = gpu_candidates(d, nt, widths, gamma, with_peaks=True)
    ws, ww, wt = oracle.boxcar_peaks(want, widths)
    assert np.array_equal(peaks[0], ws, equal_nan=True)
    assert np.array_equal(peaks[1], ww) and np.array_equal(peaks[2], wt)
    wc = oracle.boxcar_candidates(want, widths, gamma)
    got_c = as_tuples(rec)
    assert n == len(wc)
    assert [c[:3] for c in got_c] == [c[:3] for c in wc]
    assert np.array_equal(np.array([c[3] for c in got_c]), np.array([c[3] for c in wc]))


U = 2.0 ** -24


@pytest.mark.parametrize("seed", range(12))
def test_random_shape_normalised_matches_oracle(seed):
    """The normalised variant on the same random shapes (its own tiles):
    weights equal to the oracle's, float32 dedispersion within the stated
    rounding bound of the float64 oracle, and the float matched filter on the
    resulting float32 series against the oracle on the same series."""
    torch = torch_cuda()
    nchan, nsub, f_top, f_bot, tsamp, dms, g, nt, _, widths, gamma = _shape(seed)
    weighting = seed % 2
    print(f"random normalised shape {seed}: nchan {nchan} nsub {nsub} ndm {len(dms)} g {g} nt {nt} "
          f"weighting {weighting} widths {widths}", flush=True)
    sys.stdout.flush()
    freqs = synth.band_centres(f_top, f_bot, nchan)
    ref = oracle.make_plan(freqs, tsamp, dms, nsub, g=None if g == 0 else g)
    plan = tx.tx_plan(freqs, tsamp, dms, nsub, dms_per_group=g)
    n = nt + ref.overlap
    rng = np.random.default_rng(2000 + seed)
    mu = rng.uniform(60.0, 190.0, size=nchan)
    sig = rng.uniform(3.0, 30.0, size=nchan)
    x = np.clip(np.rint(mu[:, None] + sig[:, None] * rng.standard_normal((nchan, n))), 0, 255).astype(np.uint8)
    d_in = torch.from_numpy(np.ascontiguousarray(
        np.pad(x, ((0, 0), (0, (-n) % 256))))).to("cuda")
    sums = torch.empty((nchan, 4), dtype=torch.int64, device="cuda")
    tx.tx_channel_power_sums(d_in, nchan, n, sums)
    torch.cuda.synchronize()
    h = sums.cpu().numpy()
    scale, offset = tx.tx_norm_weights(h, n, weighting)
    ws_, wo_ = oracle.norm_weights(h, n, weighting)
    assert np.array_equal(scale.astype(np.float64), ws_) and np.array_equal(offset.astype(np.float64), wo_)
    out = torch.full((plan.ndm, nt), -7.0, dtype=torch.float32, device="cuda")
    tx.tx_dedisperse_norm(plan, d_in, nt, torch.from_numpy(scale).to("cuda"), torch.from_numpy(offset).to("cuda"),
                          out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = oracle.dedisperse_subband_norm(x, ref, nt, ws_, wo_)
    bound = (ref.m + ref.nsub + 1) * U * oracle.norm_abs_bound(x, ref, nt, ws_, wo_)
    assert np.all(np.abs(got.astype(np.float64) - want) <= bound)

    ndm = plan.ndm
    snr = torch.empty(ndm, dtype=torch.float64, device="cuda")
    wid = torch.empty(ndm, dtype=torch.int32, device="cuda")
    tim = torch.empty(ndm, dtype=torch.int64, device="cuda")
    raw = torch.zeros((1 << 18, 3), dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    tx.tx_candidates_f32(out, nt, widths, gamma, raw, cnt, peaks=(snr, wid, tim))
    torch.cuda.synchronize()
    Yd = got.astype(np.float64)
    es, ew, et = oracle.boxcar_peaks_float(Yd, widths)
    gs, gw, gt = snr.cpu().numpy(), wid.cpu().numpy(), tim.cpu().numpy()
    assert np.allclose(gs, es, rtol=1e-9, atol=1e-12)
    for r in range(ndm):
        if (gw[r], gt[r]) != (ew[r], et[r]):          # a near tie: the GPU's pick must be as good
            s = oracle.boxcar_snr_series_float(Yd[r], int(gw[r]))[int(gt[r])]
            assert abs(s - es[r]) <= 1e-9 * abs(es[r])
    got_c = {(c[0], c[1]): c for c in as_tuples(tx.parse_candidates(raw.cpu().numpy(), int(cnt.item())))}
    want_c = {(c[0], c[1]): c for c in oracle.boxcar_candidates_float(Yd, widths, gamma)}
    for k in set(got_c) ^ set(want_c):                # only points at the threshold may differ
        c = got_c.get(k) or want_c.get(k)
        assert abs(c[3] - gamma) < 1e-9 * gamma, c
    for k in set(got_c) & set(want_c):
        assert abs(got_c[k][3] - want_c[k][3]) <= 1e-9 * abs(want_c[k][3])


@pytest.mark.parametrize("mix", range(4))
def test_random_batch_mix_matches_oracle(mix):
    """Batches (plain and graph-captured) of five random jobs, each with its
    own plan, tile variants, widths and threshold: every job's output, peaks
    and candidates against the oracle."""
    torch = torch_cuda()
    jobs = []
    draw = 100 + 10 * mix
    while len(jobs) < 5:
        k = len(jobs)
        nchan, nsub, f_top, f_bot, tsamp, dms, g, nt, tiles, widths, gamma = _shape(draw)
        draw += 1
        freqs = synth.band_centres(f_top, f_bot, nchan)
        ref = oracle.make_plan(freqs, tsamp, dms, nsub, g=None if g == 0 else g)
        plan = tx.tx_plan(freqs, tsamp, dms, nsub, dms_per_group=g)
        plan.set_tiles(*tiles)
        if not _supported(plan, nt):
            continue                                   # refused shapes are covered by the test above
        n = nt + ref.overlap
        x = synth.uniform_u8(nchan, n, 3000 + draw)
        d_in = torch.zeros((nchan, (n + 255) // 256 * 256), dtype=torch.uint8, device="cuda")
        d_in[:, :n] = torch.from_numpy(x).to("cuda")
        y = torch.full((plan.ndm, nt + (nt & 1)), -5, dtype=torch.int32, device="cuda")   # even pitch
        peaks = (torch.empty(plan.ndm, dtype=torch.float64, device="cuda"),
                 torch.empty(plan.ndm, dtype=torch.int32, device="cuda"),
                 torch.empty(plan.ndm, dtype=torch.int64, device="cuda"))
        cands = torch.zeros((1 << 18, 3), dtype=torch.int64, device="cuda")
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
        jobs.append(dict(ref=ref, plan=plan, x=x, d_in=d_in, nt=nt, y=y, peaks=peaks, cands=cands, count=count,
                         widths=widths, gamma=gamma, tiles=tiles))
        print(f"batch mix {mix} job {k}: nchan {nchan} nsub {nsub} ndm {len(dms)} g {ref.g} nt {nt} "
              f"tiles {tiles} widths {widths}", flush=True)
    sys.stdout.flush()
    batch = tx.Batch(8, graph=bool(mix % 2))
    for j in jobs:
        batch.add(j["plan"], j["d_in"], j["nt"], j["y"], widths=j["widths"], gamma=j["gamma"], peaks=j["peaks"],
                  cands=j["cands"], count=j["count"])
    for rep in range(2):                               # a graph is captured on the first launch, replayed after
        for j in jobs:
            j["y"].fill_(-5)
            j["count"].fill_(-1)
        batch.launch()
        batch.wait()
        for j in jobs:
            nt = j["nt"]
            want = oracle.dedisperse_subband(j["x"], j["ref"], nt)
            assert np.array_equal(j["y"][:, :nt].cpu().numpy(), want)
            ws, ww, wt = oracle.boxcar_peaks(want, j["widths"])
            assert np.array_equal(j["peaks"][0].cpu().numpy(), ws, equal_nan=True)
            assert np.array_equal(j["peaks"][1].cpu().numpy(), ww)
            assert np.array_equal(j["peaks"][2].cpu().numpy(), wt)
            wc = oracle.boxcar_candidates(want, j["widths"], j["gamma"])
            n_got = int(j["count"].item())
            got_c = as_tuples(tx.parse_candidates(j["cands"].cpu().numpy(), n_got))
            assert n_got == len(wc)
            assert [c[:3] for c in got_c] == [c[:3] for c in wc]
            assert np.array_equal(np.array([c[3] for c in got_c]), np.array([c[3] for c in wc]))
    batch.close()
