"""Dedispersion plans in DM ranges with downsampling (Sec. 2.3): the HIP
downsample against the oracle's, and every range of a multi-range plan
against the oracle's sub-band dedispersion of the oracle-downsampled block."""

import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2401_13834_amd as tx
from gpu_helpers import device_block, round_up, torch_cuda

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# Lanes make 16 outputs: shapes span several lanes and rows, with ragged
# tails, a single output and a single channel.
@pytest.mark.parametrize("k", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("nchan,nt_out", [(48, 777), (256, 1024), (5, 1), (130, 33), (1, 100)])
def test_downsample_matches_oracle(k, nchan, nt_out):
    torch = torch_cuda()
    _say(f"downsample k={k} nchan={nchan} nt_out={nt_out}")
    rng = np.random.default_rng(k * 1000 + nchan * 7 + nt_out)
    x = rng.integers(0, 256, size=(nchan, k * nt_out + 5), dtype=np.uint8)
    d_in = device_block(x)
    out_pitch = round_up(nt_out, 16) + 16
    d_out = torch.full((nchan, out_pitch), 0x5A, dtype=torch.uint8, device="cuda")
    tx.tx_downsample(d_in, nchan, nt_out, k, d_out)
    got = d_out.cpu().numpy()
    assert np.array_equal(got[:, :nt_out], oracle.downsample(x, k, nt_out))
    assert np.all(got[:, nt_out:] == 0x5A)


def test_downsample_rejects_bad_arguments():
    torch = torch_cuda()
    d = torch.zeros((4, 256), dtype=torch.uint8, device="cuda")
    o = torch.zeros((4, 256), dtype=torch.uint8, device="cuda")
    with pytest.raises(tx.TxError):
        tx.tx_downsample(d, 4, 10, 3, o)          # not a power of two
    with pytest.raises(tx.TxError):
        tx.tx_downsample(d, 4, 10, 128, o)        # beyond 64
    with pytest.raises(tx.TxError):
        tx.tx_downsample(d, 4, 200, 2, o)         # input row shorter than k * nt_out


SMALL = dict(nchan=128, nsub=8, ft=1712.0, fb=856.0, tsamp=306.24e-6)
SMALL_RANGES = [(np.arange(60, dtype=np.float64) * 2.0, 1),
                (120.0 + 4.0 * np.arange(40, dtype=np.float64), 2),
                (280.0 + 8.0 * np.arange(30, dtype=np.float64), 4)]


def _ranges(freqs, tsamp, nsub, ranges):
    plans = [tx.tx_plan(freqs, tsamp * k, dms, nsub) for dms, k in ranges]
    refs = [oracle.make_plan(freqs, tsamp * k, dms, nsub) for dms, k in ranges]
    return plans, refs, tx.Ranges(plans, [k for _, k in ranges])


@pytest.mark.parametrize("nt", [4096, 1028, 4])
def test_ranges_match_oracle(nt):
    torch = torch_cuda()
    freqs = synth.band_centres(SMALL["ft"], SMALL["fb"], SMALL["nchan"])
    plans, refs, rg = _ranges(freqs, SMALL["tsamp"], SMALL["nsub"], SMALL_RANGES)
    need = rg.input_len(nt)
    assert need == max(k * (nt // k + r.overlap) for r, (_, k) in zip(refs, SMALL_RANGES))
    x = synth.uniform_u8(SMALL["nchan"], need, 51)
    d_in = device_block(x)
    outs = [torch.full((p.ndm, round_up(max(nt // k, 2), 2)), -1, dtype=torch.int32, device="cuda")
            for p, (_, k) in zip(plans, SMALL_RANGES)]
    _say(f"ranges nt={nt} input {need}")
    rg.dedisperse(d_in, nt, outs)
    torch.cuda.synchronize()
    for r, (ref, (_, k)) in enumerate(zip(refs, SMALL_RANGES)):
        want = oracle.dedisperse_subband(oracle.downsample(x, k), ref, nt // k)
        assert np.array_equal(outs[r][:, :nt // k].cpu().numpy(), want), r


def test_ranges_reject_inconsistent_plans():
    freqs = synth.band_centres(1500.0, 1100.0, 64)
    dms = np.arange(10, dtype=np.float64)
    p1 = tx.tx_plan(freqs, 1e-3, dms, 8)
    p2 = tx.tx_plan(freqs, 2e-3, dms, 8)
    p3 = tx.tx_plan(synth.band_centres(1500.0, 1000.0, 64), 2e-3, dms, 8)
    with pytest.raises(tx.TxError):
        tx.Ranges([p1, p2], [1, 3])                # factor not a power of two
    with pytest.raises(tx.TxError):
        tx.Ranges([p1, p2], [1, 4])                # sampling time is not 1e-3 * 4
    with pytest.raises(tx.TxError):
        tx.Ranges([p1, p3], [1, 2])                # different channels
    rg = tx.Ranges([p1, p2], [1, 2])
    with pytest.raises(tx.TxError):
        rg.input_len(1001)                          # not a multiple of every factor


@pytest.mark.slow
def test_ranges4096_full_size_sampled_rows():
    # The paper-scale block in three ranges: every range on sampled trial rows
    # (first, last, and a middle one) against the oracle.
    torch = torch_cuda()
    wl = synth.workload("paper-4096")
    ranges = synth.dm_ranges("ranges-4096")
    plans, refs, rg = _ranges(wl.freqs, wl.tsamp, wl.nsub, ranges)
    nt = wl.nt
    need = rg.input_len(nt)
    nchan = len(wl.freqs)
    _say(f"ranges-4096: input {nchan} x {need}")
    x = synth.pooled_normal_u8(nchan, need, wl.seed)
    d_in = device_block(x)
    outs = [torch.empty((p.ndm, nt // k), dtype=torch.int32, device="cuda") for p, (_, k) in zip(plans, ranges)]
    rg.dedisperse(d_in, nt, outs)
    torch.cuda.synchronize()
    del d_in
    for r, (ref, (dms, k)) in enumerate(zip(refs, ranges)):
        rows = [0, len(dms) // 2 + 1, len(dms) - 1]
        _say(f"ranges-4096: range {r} (k={k}) rows {rows}")
        xd = oracle.downsample(x, k)
        want = oracle.dedisperse_offsets(xd, ref.offsets[rows], nt // k)
        assert np.array_equal(outs[r][rows].cpu().numpy(), want), r
