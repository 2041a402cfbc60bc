"""tx_dedisperse_noalloc (first-stage series in the library's fixed device
scratch, no allocation) against tx_dedisperse, through the C ABI: bit-exact
on two calls in a row, the second with a smaller block, on a plan whose
series need several chunks and on one that needs one; replayed from a
captured HIP graph; and the error for a plan whose series do not fit."""

import sys

import numpy as np
import pytest

import synth
import paper_2401_13834_amd as tx
from gpu_helpers import device_block, round_up, torch_cuda

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(torch, plan, d_in, nt, fill=-9):
    """(tx_dedisperse output, tx_dedisperse_noalloc output) of one block,
    with a few columns past nt that neither may write."""
    want = torch.full((plan.ndm, round_up(nt, 2) + 6), fill, dtype=torch.int32, device="cuda")
    got = torch.full_like(want, fill)
    tx.tx_dedisperse(plan, d_in, nt, want)
    tx.tx_dedisperse_noalloc(plan, d_in, nt, got)
    torch.cuda.synchronize()
    return want, got


def test_noalloc_equals_dedisperse_paper_scale_two_calls():
    torch = torch_cuda()
    wl = synth.workload("paper-4096")
    plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    assert plan.ws_size(wl.nt) > tx.TX_NOALLOC_SCRATCH_BYTES      # several chunks
    d_in = synth.device_normal_u8(torch, plan.nchan, round_up(wl.nt + plan.overlap, 256), 21)
    for nt in (wl.nt, 20011):                                   # then a smaller, ragged block
        _say(f"noalloc paper-4096 nt={nt}")
        want, got = _pair(torch, plan, d_in, nt)
        assert torch.equal(got, want)
        assert bool((got[:, nt:] == -9).all())
        del want, got
    torch.cuda.empty_cache()


def test_noalloc_equals_dedisperse_small_two_calls():
    torch = torch_cuda()
    freqs = synth.band_centres(1712.0, 856.0, 256)
    plan = tx.tx_plan(freqs, 306.24e-6, np.arange(128) * 4.0, 16)
    assert plan.ws_size(8192) <= tx.TX_NOALLOC_SCRATCH_BYTES     # one chunk
    x = synth.uniform_u8(256, 8192 + plan.overlap, 5)
    d_in = device_block(x)
    for nt in (8192, 3001):
        _say(f"noalloc plain-256 nt={nt}")
        want, got = _pair(torch, plan, d_in, nt)
        assert torch.equal(got, want)


def test_noalloc_replays_from_a_captured_graph():
    torch = torch_cuda()
    freqs = synth.band_centres(1712.0, 856.0, 1024)
    plan = tx.tx_plan(freqs, 153.12e-6, np.linspace(0.0, 1000.0, 512), 64)
    nt = 16384
    d_in = synth.device_normal_u8(torch, plan.nchan, round_up(nt + plan.overlap, 256), 31)
    want = torch.empty((plan.ndm, nt), dtype=torch.int32, device="cuda")
    got = torch.empty_like(want)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tx.tx_dedisperse_noalloc(plan, d_in, nt, got, stream=s)     # eager first use
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        tx.tx_dedisperse_noalloc(plan, d_in, nt, got, stream=s)
    for rep in range(3):
        _say(f"noalloc graph replay {rep}")
        d_in.copy_(synth.device_normal_u8(torch, plan.nchan, d_in.shape[1], 40 + rep))
        got.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        tx.tx_dedisperse(plan, d_in, nt, want)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
    del g


def test_noalloc_rejects_a_plan_whose_series_do_not_fit():
    torch = torch_cuda()
    freqs = synth.band_centres(1712.0, 856.0, 1024)
    # one trial per coarse group: 2048 groups x 64 sub-bands of series
    plan = tx.tx_plan(freqs, 153.12e-6, np.linspace(0.0, 1000.0, 2048), 64, dms_per_group=1)
    nt = 4096
    d_in = torch.zeros((plan.nchan, round_up(nt + plan.overlap, 256)), dtype=torch.uint8, device="cuda")
    out = torch.full((plan.ndm, nt), -4, dtype=torch.int32, device="cuda")
    with pytest.raises(tx.TxError) as err:
        tx.tx_dedisperse_noalloc(plan, d_in, nt, out)
    assert err.value.status == tx.TX_ENOTSUP
    assert "scratch" in str(err.value)
    torch.cuda.synchronize()
    assert bool((out == -4).all())                               # nothing was queued
