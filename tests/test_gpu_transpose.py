"""Time-major ingest (the "transpose" step of Sec. 2.3, Fig.
"dedispersion_flow"): the HIP transpose against the oracle's channel_rows,
and time-major stream pushes / batches against channel-major ones and the
oracle on the concatenated input."""

import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2401_13834_amd as tx
from gpu_helpers import round_up, torch_cuda

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _time_major(torch, x_tf, pitch, device=True):
    nt, nchan = x_tf.shape
    t = torch.zeros((max(nt, 1), pitch), dtype=torch.uint8)
    t[:nt, :nchan] = torch.from_numpy(np.ascontiguousarray(x_tf))
    return t.to("cuda") if device else t.pin_memory()


# Tiles are 128 channels x 128 samples: shapes span several tiles with ragged
# channel and time tails, a single channel, a single sample, and exact tiles.
SHAPES = [(4096, 1000), (48, 777), (130, 129), (1, 17), (16, 16), (256, 4099), (17, 1), (128, 128), (200, 300)]


@pytest.mark.parametrize("nchan,nt", SHAPES)
def test_transpose_matches_oracle(nchan, nt):
    torch = torch_cuda()
    _say(f"transpose nchan={nchan} nt={nt}")
    rng = np.random.default_rng(nchan * 7919 + nt)
    x_tf = rng.integers(0, 256, size=(nt, nchan), dtype=np.uint8)
    tf_pitch = round_up(nchan, 16) + 16                    # wider than the channels
    d_tf = _time_major(torch, x_tf, tf_pitch)
    ft_pitch = round_up(nt, 16) + 32
    d_ft = torch.full((nchan, ft_pitch), 0xA5, dtype=torch.uint8, device="cuda")
    tx.tx_transpose_tf(d_tf, nchan, nt, d_ft)
    got = d_ft.cpu().numpy()
    assert np.array_equal(got[:, :nt], oracle.channel_rows(x_tf, nchan))
    assert np.all(got[:, nt:] == 0xA5)                     # bytes past nt untouched


def test_transpose_paper_scale_block():
    # A paper-scale block: 4096 channels x 65536 + overlap samples (recorded
    # time-major), the size one served block ingests.
    torch = torch_cuda()
    nchan, nt = 4096, 65536 + 4099
    _say(f"transpose full size {nchan} x {nt}")
    gen = torch.Generator(device="cuda").manual_seed(5)
    d_tf = torch.randint(0, 256, (nt, nchan), dtype=torch.uint8, device="cuda", generator=gen)
    d_ft = torch.empty((nchan, round_up(nt, 256)), dtype=torch.uint8, device="cuda")
    tx.tx_transpose_tf(d_tf, nchan, nt, d_ft)
    torch.cuda.synchronize()
    x_tf = d_tf.cpu().numpy()
    assert np.array_equal(d_ft[:, :nt].cpu().numpy(), oracle.channel_rows(x_tf, nchan))


def test_transpose_rejects_bad_arguments():
    torch = torch_cuda()
    d = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    o = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(tx.TxError):
        tx.tx_transpose_tf(d[:, 1:], 32, 32, o)             # misaligned input
    with pytest.raises(tx.TxError):
        tx.tx_transpose_tf(d, 65, 32, o)                    # pitch below nchan
    with pytest.raises(tx.TxError):
        tx.tx_transpose_tf(d, 32, 65, o)                    # output pitch below nt


def _plan_pair(nchan, nsub, ndm, dmmax, ft=1712.0, fb=856.0, ts=306.24e-6):
    freqs = synth.band_centres(ft, fb, nchan)
    dms = np.linspace(0.0, dmmax, ndm)
    return oracle.make_plan(freqs, ts, dms, nsub), tx.tx_plan(freqs, ts, dms, nsub)


def test_time_major_stream_equals_concatenated_block():
    torch = torch_cuda()
    ref, plan = _plan_pair(128, 8, 60, 400.0)
    O = ref.overlap
    sizes = [O // 3, O // 3, O // 2, 3000, 1, 4097, 2500, 777]
    total = sum(sizes)
    x = synth.uniform_u8(128, total, 41)                   # channel rows (the oracle's input)
    x_tf = np.ascontiguousarray(x.T)                       # as recorded
    st = tx.Stream(plan, max(sizes))
    outs = []
    pos = 0
    for k, n in enumerate(sizes):
        blk = _time_major(torch, x_tf[pos:pos + n], 144, device=bool(k % 2))
        d_out = torch.full((plan.ndm, round_up(max(n, 2), 2)), -1, dtype=torch.int32, device="cuda")
        got = st.push_tf(blk, n, d_out)
        torch.cuda.synchronize()
        outs.append(d_out[:, :got].cpu().numpy())
        pos += n
        _say(f"push_tf {k}: {n} -> {got}")
    y = np.concatenate(outs, axis=1)
    assert y.shape[1] == total - O
    want = oracle.dedisperse_subband(oracle.channel_rows(x_tf, 128), ref, total - O)
    assert np.array_equal(y, want)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_of_time_major_streams_equals_channel_major(graph):
    torch = torch_cuda()
    specs = [(128, 8, 60, 400.0), (64, 4, 30, 250.0), (96, 12, 45, 600.0)]
    pairs = [_plan_pair(*sp) for sp in specs]
    block = 2000
    nblocks = 5
    xs = [synth.uniform_u8(sp[0], block * nblocks, 400 + k) for k, sp in enumerate(specs)]
    tf = [tx.Stream(p, block) for _, p in pairs]
    cm = [tx.Stream(p, block) for _, p in pairs]
    batch = tx.Batch(4, graph=graph)
    s = torch.cuda.Stream()
    outs_tf = [[] for _ in specs]
    outs_cm = [[] for _ in specs]
    with torch.cuda.stream(s):
        for k in range(nblocks):
            _say(f"time-major batch graph={graph} block {k}")
            batch.clear()
            blocks_tf = [_time_major(torch, np.ascontiguousarray(x[:, k * block:(k + 1) * block].T),
                                     round_up(x.shape[0], 16), device=(q == 1)) for q, x in enumerate(xs)]
            blocks_cm = [torch.from_numpy(np.ascontiguousarray(x[:, k * block:(k + 1) * block])).to("cuda")
                         for x in xs]
            d_tf = [torch.empty((p.ndm, block), dtype=torch.int32, device="cuda") for _, p in pairs]
            for q in range(len(specs)):
                batch.add_stream_tf(tf[q], blocks_tf[q], block, d_tf[q])
            batch.launch(s)
            n_tf = [batch.stream_output(q) for q in range(len(specs))]
            for q in range(len(specs)):
                d_cm = torch.empty((pairs[q][1].ndm, block), dtype=torch.int32, device="cuda")
                n_cm = cm[q].push(blocks_cm[q], block, d_cm, stream=s)
                assert n_cm == n_tf[q]
                s.synchronize()
                outs_tf[q].append(d_tf[q][:, :n_tf[q]].cpu().numpy())
                outs_cm[q].append(d_cm[:, :n_cm].cpu().numpy())
    for q, (ref, _) in enumerate(pairs):
        yt = np.concatenate(outs_tf[q], axis=1)
        yc = np.concatenate(outs_cm[q], axis=1)
        assert np.array_equal(yt, yc)
        n = yt.shape[1]
        assert n == block * nblocks - ref.overlap
        assert np.array_equal(yt, oracle.dedisperse_subband(xs[q], ref, n))
