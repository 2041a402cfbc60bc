"""Channel masks and statistics (Sec. 2.2): exact per-channel power sums on the
GPU against the oracle, dedispersion with dropped channels against the
oracle on zeroed rows (stateless, streams, batches, every tile variant), and
the skewness-kurtosis mask end to end."""

import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2401_13834_amd as tx
from gpu_helpers import device_block, gpu_dedisperse, torch_cuda

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("nchan,nt", [(64, 100000), (3, 1), (130, 16385), (1, 33000), (4096, 4096)])
def test_power_sums_match_oracle(nchan, nt):
    torch = torch_cuda()
    _say(f"power sums {nchan} x {nt}")
    x = synth.uniform_u8(nchan, nt, nchan + nt)
    d_in = device_block(x)
    sums = torch.full((nchan, 4), -1, dtype=torch.int64, device="cuda")
    tx.tx_channel_power_sums(d_in, nchan, nt, sums)
    got = sums.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, oracle.channel_power_sums(x).astype(np.uint64))


def _plan_pair(nchan, nsub, ndm, dmmax, ft=1712.0, fb=856.0, ts=306.24e-6):
    freqs = synth.band_centres(ft, fb, nchan)
    dms = np.linspace(0.0, dmmax, ndm)
    return oracle.make_plan(freqs, ts, dms, nsub), tx.tx_plan(freqs, ts, dms, nsub)


def test_mask_round_trip_and_clear():
    _, plan = _plan_pair(64, 8, 20, 100.0)
    assert np.all(plan.get_mask() == 1)
    m = np.ones(64, dtype=np.uint8)
    m[[1, 7, 63]] = 0
    plan.set_mask(m)
    assert np.array_equal(plan.get_mask(), m)
    plan.set_mask(None)
    assert np.all(plan.get_mask() == 1)


def test_masked_dedispersion_every_variant():
    torch_cuda()
    ref, plan = _plan_pair(256, 16, 128, 508.0)
    nt = 5000
    x = synth.uniform_u8(256, nt + ref.overlap, 61)
    rng = np.random.default_rng(62)
    mask = (rng.random(256) > 0.2).astype(np.uint8)
    mask[0] = 0                                   # the reference channel too
    plan.set_mask(mask)
    want = oracle.dedisperse_subband(x * mask[:, None], ref, nt)
    d = device_block(x)
    n1 = len(tx.tx_tile_variants(1))
    for s1 in range(n1):
        _say(f"masked variant {s1}")
        plan.set_tiles(s1, 0, -1, 0)
        got = gpu_dedisperse(plan, x, nt, d_in=d)
        assert np.array_equal(got[:, :nt], want), s1
    plan.set_tiles()
    plan.set_mask(None)
    got = gpu_dedisperse(plan, x, nt, d_in=d)
    assert np.array_equal(got[:, :nt], oracle.dedisperse_subband(x, ref, nt))


@pytest.mark.parametrize("graph", [False, True])
def test_masked_streams_and_batches(graph):
    torch = torch_cuda()
    ref, plan = _plan_pair(128, 8, 60, 400.0)
    mask = np.ones(128, dtype=np.uint8)
    mask[10:20] = 0
    mask[77] = 0
    plan.set_mask(mask)
    block, nblocks = 2000, 5
    x = synth.uniform_u8(128, block * nblocks, 63)
    st_single = tx.Stream(plan, block)
    st_batch = tx.Stream(plan, block)
    batch = tx.Batch(2, graph=graph)
    s = torch.cuda.Stream()
    out_s, out_b = [], []
    with torch.cuda.stream(s):
        for k in range(nblocks):
            _say(f"masked stream/batch graph={graph} block {k}")
            blk = torch.from_numpy(np.ascontiguousarray(x[:, k * block:(k + 1) * block])).to("cuda")
            d_s = torch.empty((plan.ndm, block), dtype=torch.int32, device="cuda")
            d_b = torch.empty((plan.ndm, block), dtype=torch.int32, device="cuda")
            n_s = st_single.push(blk, block, d_s, stream=s)
            batch.clear()
            batch.add_stream(st_batch, blk, block, d_b)
            batch.launch(s)
            n_b = batch.stream_output(0)
            s.synchronize()
            assert n_s == n_b
            out_s.append(d_s[:, :n_s].cpu().numpy())
            out_b.append(d_b[:, :n_b].cpu().numpy())
    ys, yb = np.concatenate(out_s, axis=1), np.concatenate(out_b, axis=1)
    assert np.array_equal(ys, yb)
    assert np.array_equal(ys, oracle.dedisperse_subband(x * mask[:, None], ref, ys.shape[1]))


def test_skf_mask_end_to_end():
    # A block with planted narrow-band RFI: GPU power sums -> host mask ->
    # plan mask -> dedispersion, against the oracle at every step.
    torch = torch_cuda()
    ref, plan = _plan_pair(256, 16, 100, 400.0)
    nt = 8192
    n = nt + ref.overlap
    x = synth.normal_u8(256, n, 64)
    x[12] = 128
    x[12, ::61] = 255                                # impulsive
    x[100] = np.clip(x[100].astype(np.int64) + (np.arange(n) % 40 < 4) * 100, 0, 255).astype(np.uint8)
    x[200] = 3                                       # dead channel
    d = device_block(x)
    sums = torch.empty((256, 4), dtype=torch.int64, device="cuda")
    tx.tx_channel_power_sums(d, 256, n, sums)
    s_host = sums.cpu().numpy()
    w_sums = oracle.channel_power_sums(x)
    assert np.array_equal(s_host.view(np.uint64), w_sums.astype(np.uint64))
    mask = tx.tx_skf_mask(s_host, n, 5.0)
    w_mask = oracle.skf_mask(w_sums, n, 5.0)
    assert np.array_equal(mask, w_mask)
    assert {12, 100, 200} <= set(np.nonzero(mask == 0)[0].tolist())
    plan.set_mask(mask)
    got = gpu_dedisperse(plan, x, nt, d_in=d)
    assert np.array_equal(got[:, :nt], oracle.dedisperse_subband(x * w_mask[:, None], ref, nt))
