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
