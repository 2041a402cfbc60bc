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
    """A captured batch graph holds persistent launches of the kernel classes
    (tile variant, trials per second-stage workgroup) and LDS sizes it was
    captured with: any number and size of jobs of those classes replays; a
    job needing a class it lacks is refused before anything is queued, and a
    reservation made before capture adds the class."""
    torch = torch_cuda()
    freqs = synth.band_centres(1712.0, 856.0, 64)
    dms = np.linspace(0.0, 300.0, 40)
    ref = oracle.make_plan(freqs, 306.24e-6, dms, 8)
    plan = tx.tx_plan(freqs, 306.24e-6, dms, 8)
    ref1 = oracle.make_plan(freqs, 306.24e-6, dms, 8, g=1)
    plan1 = tx.tx_plan(freqs, 306.24e-6, dms, 8, dms_per_group=1)    # 1 trial per second-stage workgroup
    assert plan.g > 1
    small, big = 2000, 6000
    x = synth.uniform_u8(64, big + max(ref.overlap, ref1.overlap), 79)
    d_in = torch.zeros((64, round_up(x.shape[1], 256)), dtype=torch.uint8, device="cuda")
    d_in[:, :x.shape[1]] = torch.from_numpy(x).to("cuda")
    y = torch.zeros((plan.ndm, big), dtype=torch.int32, device="cuda")
    y1 = torch.zeros((plan.ndm, big), dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    b = tx.Batch(3, graph=True)
    b.add(plan, d_in, small, y)
    with torch.cuda.stream(s):
        b.launch(s)                                     # captured with one small job
        b.clear()
        b.add(plan, d_in, big, y)                       # more tiles: same kernels, replays
        b.add(plan, d_in, small, y1)
        b.launch(s)
        b.wait()
    assert np.array_equal(y[:, :big].cpu().numpy(), oracle.dedisperse_subband(x, ref, big))
    assert np.array_equal(y1[:, :small].cpu().numpy(), oracle.dedisperse_subband(x, ref, small))
    with torch.cuda.stream(s):
        b.clear()
        b.add(plan1, d_in, small, y1)
        with pytest.raises(tx.TxError) as err:
            b.launch(s)                                 # a second-stage class the graph lacks
        assert err.value.status == tx.TX_ESTATE
        b.close()
        r = tx.Batch(2, graph=True)
        r.reserve(plan1, 0, big, 1)
        r.add(plan, d_in, small, y)
        r.launch(s)
        r.clear()
        r.add(plan1, d_in, big, y1)
        r.add(plan, d_in, big, y)
        r.launch(s)
        s.synchronize()
        r.close()
    assert np.array_equal(y[:, :big].cpu().numpy(), oracle.dedisperse_subband(x, ref, big))
    assert np.array_equal(y1[:, :big].cpu().numpy(), oracle.dedisperse_subband(x, ref1, big))


@pytest.mark.parametrize("graph", [False, True])
def test_batch_jobs_keep_their_own_tiles(graph):
    """Jobs whose plans use different tile variants (as per-shape autotuning
    leaves them) run in one batch, each in its own variant's launch, and
    equal the oracle."""
    torch = torch_cuda()
    n1 = len(tx.tx_tile_variants(1))
    n2 = len(tx.tx_tile_variants(2))
    freqs = synth.band_centres(1712.0, 856.0, 128)
    jobs = []
    for k in range(5):
        dms = np.linspace(0.0, 200.0 + 100.0 * k, 50 + 10 * k)
        ref = oracle.make_plan(freqs, 306.24e-6, dms, 8)
        plan = tx.tx_plan(freqs, 306.24e-6, dms, 8)
        plan.set_tiles(k % n1, 0, (2 * k + 1) % n2, 0)
        nt = 3000 + 700 * k
        x = synth.uniform_u8(128, nt + ref.overlap, 90 + k)
        d_in = torch.zeros((128, round_up(x.shape[1], 256)), dtype=torch.uint8, device="cuda")
        d_in[:, :x.shape[1]] = torch.from_numpy(x).to("cuda")
        y = torch.full((plan.ndm, nt), -1, dtype=torch.int32, device="cuda")
        jobs.append((ref, plan, x, d_in, y, nt))
    b = tx.Batch(len(jobs), graph=graph)
    for ref, plan, x, d_in, y, nt in jobs:
        b.add(plan, d_in, nt, y)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(2):
            for job in jobs:
                job[4].fill_(-1)
            b.launch(s)
            b.wait()
            for ref, plan, x, d_in, y, nt in jobs:
                assert np.array_equal(y.cpu().numpy(), oracle.dedisperse_subband(x, ref, nt))
    b.close()
