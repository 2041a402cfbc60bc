"""Host-side checks of libtx: the library loads and exports every declared
entry point, and the host plan (delay tables, groups, offsets, overlap)
equals the oracle's bit for bit.  No device calls."""

import os
import re

import numpy as np
import pytest

import oracle
import synth
import paper_2401_13834_amd as tx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tx_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = tx.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(tx.exported_names()) | set(dir(L))
    assert L.tx_version().decode().startswith("libtx")
    assert L.tx_status_str(-1).decode() == "TX_EINVAL"


WORKLOADS = ["plain-256", "paper-4096", "served-4096", "octave-8192"]


@pytest.mark.parametrize("name", WORKLOADS)
def test_host_plan_equals_oracle(name):
    wl = synth.workload(name)
    ref = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    p = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub, host_only=True)
    assert (p.nsub, p.g, p.ngroups, p.overlap) == (ref.nsub, ref.g, ref.ngroups, ref.overlap)
    assert p.max_extent == int(ref.extent.max())
    assert p.on_device == 0
    t = p.tables()
    assert np.array_equal(t["coarse_chan"], ref.d_coarse_chan)
    assert np.array_equal(t["coarse_sub"], ref.d_coarse_sub)
    assert np.array_equal(t["fine_sub"], ref.d_fine_sub)
    assert np.array_equal(t["extent"], ref.extent)
    if ref.ndm * ref.nchan <= 16 * 1024 * 1024:
        assert np.array_equal(p.offsets(), ref.offsets)
    for dm in (0.0, float(wl.dms[len(wl.dms) // 3]), float(wl.dms[-1])):
        assert np.array_equal(p.delays(dm), oracle.delay_samples(dm, wl.freqs, ref.fref, wl.tsamp))


@pytest.mark.parametrize("seed", range(8))
def test_host_plan_random_shapes_equal_oracle(seed):
    rng = np.random.default_rng(seed)
    nsub = int(rng.choice([1, 2, 3, 4, 8]))
    m = int(rng.integers(1, 40))
    nchan = nsub * m
    freqs = rng.uniform(300.0, 2000.0, nchan)          # any channel order
    ndm = int(rng.integers(1, 60))
    dms = np.sort(rng.uniform(0.0, 2000.0, ndm))
    dms[rng.random(ndm) < 0.1] = 0.0
    dms = np.sort(dms)
    tsamp = float(rng.uniform(5e-5, 1e-3))
    g = int(rng.choice([0, 1, 2, 5, 1000]))
    ref = oracle.make_plan(freqs, tsamp, dms, nsub, g=None if g == 0 else g)
    p = tx.tx_plan(freqs, tsamp, dms, nsub, dms_per_group=g, host_only=True)
    assert (p.g, p.ngroups, p.overlap) == (ref.g, ref.ngroups, ref.overlap)
    assert np.array_equal(p.offsets(), ref.offsets)
    assert np.array_equal(p.tables()["extent"], ref.extent)


@pytest.mark.parametrize("name", ["paper-4096", "batched-0", "batched-1", "batched-2", "batched-5"])
def test_automatic_subband_count_minimises_weighted_additions(name):
    """nsub = 0: the divisor of nchan (at most 256 channels per sub-band) that
    minimises N_c * nchan + 2.5 * ndm * nsub, as documented in the header."""
    if name.startswith("batched-"):
        wl = synth.batched_beams()[int(name.split("-")[1])]
    else:
        wl = synth.workload(name)
    p = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, 0, host_only=True)
    nchan, ndm = len(wl.freqs), len(wl.dms)

    def cost(ns):
        g = oracle.group_size_rule(wl.freqs, ns, ndm)
        return -(-ndm // g) * nchan + 2.5 * ndm * ns

    cands = [ns for ns in range(1, nchan + 1) if nchan % ns == 0 and nchan // ns <= 256]
    assert p.nsub in cands
    assert cost(p.nsub) == min(cost(ns) for ns in cands)


def _status(fn):
    with pytest.raises(tx.TxError) as e:
        fn()
    return e.value.status


def test_plan_argument_errors():
    f = synth.band_centres(1712, 856, 64)
    d = np.arange(10) * 5.0
    assert _status(lambda: tx.tx_plan(f, 1e-4, d, 7, host_only=True)) == -1          # nsub does not divide
    assert _status(lambda: tx.tx_plan(np.tile(f, 8), 1e-4, d, 1, host_only=True)) == -1  # 512 chans per sub-band
    assert _status(lambda: tx.tx_plan(f, 0.0, d, 8, host_only=True)) == -1
    assert _status(lambda: tx.tx_plan(f, 1e-4, d[::-1], 8, host_only=True)) == -1     # decreasing
    assert _status(lambda: tx.tx_plan(f, 1e-4, -d, 8, host_only=True)) == -1
    assert _status(lambda: tx.tx_plan(f, 1e-4, np.array([]), 8, host_only=True)) == -1
    bad = f.copy()
    bad[3] = np.nan
    assert _status(lambda: tx.tx_plan(bad, 1e-4, d, 8, host_only=True)) == -1
    assert _status(lambda: tx.tx_plan(f * 0.01, 1e-7, d * 1e4, 8, host_only=True)) == -5  # delay overflow


def test_device_calls_on_host_only_plan_are_refused():
    f = synth.band_centres(1712, 856, 64)
    p = tx.tx_plan(f, 1e-4, np.arange(10) * 5.0, 8, host_only=True)
    L = tx.lib()
    st = L.tx_dedisperse(p.handle, 16, 4096, 8, 16, 8, None)
    assert st == -4
    with pytest.raises(tx.TxError):
        p.delays(-1.0)


def test_resolved_tiles():
    # Defaults resolve to real variant indices and LDS sizes; an explicit
    # choice comes back as set, its LDS raised to what the rows need.
    wl = synth.workload("paper-4096")
    p = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub, host_only=True)
    assert p.get_tiles() == (-1, 0, -1, 0)
    s1, l1, s2, l2 = p.resolved_tiles(wl.nt)
    assert 0 <= s1 < len(tx.tx_tile_variants(1)) and 0 <= s2 < len(tx.tx_tile_variants(2))
    assert l1 > 0 and l2 > 0
    p.set_tiles(0, 1024, 0, 1024)
    r = p.resolved_tiles(wl.nt)
    assert r[0] == 0 and r[2] == 0 and r[1] > 1024 and r[3] > 1024
    with pytest.raises(tx.TxError):
        p.resolved_tiles(-1)


def test_tune_cache_roundtrip(tmp_path):
    from paper_2401_13834_amd import tune
    f = synth.band_centres(1712.0, 856.0, 64)
    d = np.linspace(0.0, 300.0, 40)
    k1 = tune.shape_key(f, 306.24e-6, d, 8, 3000, "dev")
    assert k1 == tune.shape_key(f.copy(), 306.24e-6, d.copy(), 8, 3000, "dev")
    assert k1 != tune.shape_key(f, 306.24e-6, d, 8, 3001, "dev")
    assert k1 != tune.shape_key(f, 306.24e-6, d * 1.0000001, 8, 3000, "dev")
    path = str(tmp_path / "c" / "tiles.json")
    assert tune.load(path) == {}
    tune.save({k1: {"tiles": [3, 32768, 1, 32768], "ms": 1.5}}, path)
    assert tune.load(path)[k1]["tiles"] == [3, 32768, 1, 32768]
    assert tune.nsub_candidates(4096) == [16, 32, 64, 128, 256, 512, 1024, 2048, 4096]
    assert all(4096 % n == 0 and 4096 // n <= 256 for n in tune.nsub_candidates(4096))


def test_skf_mask_host_function_matches_oracle():
    # tx_skf_mask is host code: the C decision from power sums equals the
    # oracle's on random channel statistics, including planted outliers and a
    # zero-variance channel.
    import oracle
    import synth
    rng = np.random.default_rng(40)
    for trial in range(20):
        nchan, nt = int(rng.integers(3, 200)), int(rng.integers(2, 5000))
        x = synth.normal_u8(nchan, nt, 100 + trial)
        if nchan > 5:
            x[2] = 9
            x[4, ::7] = 250
        sums = oracle.channel_power_sums(x)
        want = oracle.skf_mask(sums, nt, 3.5)
        got = tx.tx_skf_mask(sums.astype(np.uint64), nt, 3.5)
        assert np.array_equal(got, want), trial


@pytest.mark.parametrize("weighting", [0, 1])
def test_norm_weights_host_call_equals_oracle(weighting):
    """tx_norm_weights (host code) gives the oracle's float32 weights bit for
    bit, including a zero-variance channel and very unequal channels."""
    rng = np.random.default_rng(5 + weighting)
    nchan, n = 40, 3001
    mu = rng.uniform(20.0, 230.0, size=nchan)
    sig = rng.uniform(0.3, 60.0, size=nchan)
    x = np.clip(np.rint(mu[:, None] + sig[:, None] * rng.standard_normal((nchan, n))), 0, 255).astype(np.uint8)
    x[7] = 42
    sums = oracle.channel_power_sums(x)
    scale, offset = tx.tx_norm_weights(sums, n, weighting)
    ws, wo = oracle.norm_weights(sums, n, weighting)
    assert np.array_equal(scale.astype(np.float64), ws) and np.array_equal(offset.astype(np.float64), wo)
    assert scale[7] == 0.0 and offset[7] == 0.0
    with pytest.raises(tx.TxError):
        tx.tx_norm_weights(sums, n, 2)


def test_binding_refuses_tensors_of_the_wrong_type():
    """The binding passes base pointers and row pitches in elements of the
    declared type, so a tensor of another type (say an int64 DM x time array
    given to the int32 boxcar) or with strided rows is refused before any
    library call."""
    torch = pytest.importorskip("torch")
    widths = [1, 2, 4]
    snr = torch.empty(2, dtype=torch.float64)
    wid = torch.empty(2, dtype=torch.int32)
    tim = torch.empty(2, dtype=torch.int64)
    with pytest.raises(TypeError):
        tx.tx_boxcar_snr(torch.zeros((2, 16), dtype=torch.int64), 16, widths, snr, wid, tim)
    with pytest.raises(TypeError):
        tx.tx_boxcar_snr_f32(torch.zeros((2, 16), dtype=torch.float64), 16, widths, snr, wid, tim)
    with pytest.raises(TypeError):
        tx.tx_boxcar_snr(torch.zeros((2, 16), dtype=torch.int32), 16, widths, snr.float(), wid, tim)
    with pytest.raises(TypeError):
        tx.tx_candidates(torch.zeros((2, 16), dtype=torch.int32), 16, widths, 6.0,
                         torch.zeros((4, 3), dtype=torch.int64), torch.zeros(1, dtype=torch.int32))
    with pytest.raises(ValueError):
        tx.tx_boxcar_snr(torch.zeros((16, 2), dtype=torch.int32).t(), 16, widths, snr, wid, tim)
    with pytest.raises(TypeError):
        tx.tx_dedisperse(None, torch.zeros((4, 64), dtype=torch.int32), 16, torch.zeros((4, 16), dtype=torch.int32))
    with pytest.raises(TypeError):
        tx.tx_channel_power_sums(torch.zeros((4, 64), dtype=torch.uint8), 4, 64, torch.zeros((4, 4), dtype=torch.int32))
