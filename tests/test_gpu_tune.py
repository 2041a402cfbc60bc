"""Autotuner (tile variants measured on the device, sub-band count search,
cache) and graph capacity of batches: tuned plans still match the oracle."""

import numpy as np
import pytest

import oracle
import synth
import paper_2401_13834_amd as tx
from paper_2401_13834_amd import tune
from gpu_helpers import gpu_dedisperse, round_up, torch_cuda

pytestmark = pytest.mark.gpu


def test_autotune_sets_tiles_and_keeps_output():
    torch_cuda()
    wl = synth.workload("plain-256")
    ref = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    assert plan.get_tiles()[0] == -1
    ms = plan.autotune(wl.nt, effort=1)
    assert ms > 0.0
    s1, l1, s2, l2 = plan.get_tiles()
    assert 0 <= s1 < len(tx.tx_tile_variants(1)) and 0 <= s2 < len(tx.tx_tile_variants(2))
    assert l1 > 0 and l2 > 0
    x = synth.uniform_u8(256, wl.nt + ref.overlap, 77)
    assert np.array_equal(gpu_dedisperse(plan, x, wl.nt), oracle.dedisperse_subband(x, ref, wl.nt))


def test_tune_cache_and_nsub_search(tmp_path):
    torch_cuda()
    path = str(tmp_path / "tiles.json")
    freqs = synth.band_centres(1712.0, 856.0, 128)
    tsamp = 306.24e-6
    dms = np.linspace(0.0, 400.0, 60)
    nt = 4000
    plan = tx.tx_plan(freqs, tsamp, dms, 8)
    tiles, ms = tune.tune_tiles(plan, freqs, tsamp, dms, nt, effort=0, path=path)
    assert ms is not None and ms > 0
    plan2 = tx.tx_plan(freqs, tsamp, dms, 8)
    tiles2, ms2 = tune.tune_tiles(plan2, freqs, tsamp, dms, nt, effort=0, path=path)
    assert ms2 is None and tuple(tiles2) == tuple(tiles) and plan2.get_tiles() == tuple(tiles)
    best, times = tune.plan_autotuned(freqs, tsamp, dms, nt, nsubs=[4, 8, 16], effort=0, path=path)
    assert set(times) == {4, 8, 16} and best.nsub in times
    assert times[best.nsub] == min(times.values())
    ref = oracle.make_plan(freqs, tsamp, dms, best.nsub)
    assert ref.g == best.g
    x = synth.uniform_u8(128, nt + ref.overlap, 78)
    assert np.array_equal(gpu_dedisperse(best, x, nt), oracle.dedisperse_subband(x, ref, nt))
    again, _ = tune.plan_autotuned(freqs, tsamp, dms, nt, nsubs=[4, 8, 16], effort=0, path=path)
    assert again.nsub == best.nsub


def test_graph_batch_capacity_is_checked():
    torch = torch_cuda()
    freqs = synth.band_centres(1712.0, 856.0, 64)
    dms = np.linspace(0.0, 300.0, 40)
    ref = oracle.make_plan(freqs, 306.24e-6, dms, 8)
    plan = tx.tx_plan(freqs, 306.24e-6, dms, 8)
    small, big = 2000, 6000
    x = synth.uniform_u8(64, big + ref.overlap, 79)
    d_in = torch.zeros((64, round_up(big + ref.overlap, 256)), dtype=torch.uint8, device="cuda")
    d_in[:, :x.shape[1]] = torch.from_numpy(x).to("cuda")
    y = torch.zeros((plan.ndm, big), dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    b = tx.Batch(2, graph=True)
    b.add(plan, d_in, small, y)
    with torch.cuda.stream(s):
        b.launch(s)                                     # captured for `small` outputs
        b.clear()
        b.add(plan, d_in, big, y)
        with pytest.raises(tx.TxError) as err:
            b.launch(s)                                 # more tiles than the graph holds
        assert err.value.status == tx.TX_ESTATE
        b.close()
        # a reserved graph takes the larger job
        r = tx.Batch(2, graph=True)
        r.reserve(plan, 0, big, 1)
        r.add(plan, d_in, small, y)
        r.launch(s)
        r.clear()
        r.add(plan, d_in, big, y)
        r.launch(s)
        s.synchronize()
        r.close()
    assert np.array_equal(y[:, :big].cpu().numpy(), oracle.dedisperse_subband(x, ref, big))
