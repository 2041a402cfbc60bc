"""Streams (device-resident overlap history) and batches (many uneven beams in
persistent launches, optionally a replayed HIP graph), against the oracle."""

import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2401_13834_amd as tx
from gpu_helpers import as_tuples, device_block, round_up, torch_cuda

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _plan_pair(nchan, nsub, ndm, dmmax, ft=1712.0, fb=856.0, ts=306.24e-6):
    freqs = synth.band_centres(ft, fb, nchan)
    dms = np.linspace(0.0, dmmax, ndm)
    return oracle.make_plan(freqs, ts, dms, nsub), tx.tx_plan(freqs, ts, dms, nsub)


def test_stream_equals_concatenated_block():
    torch = torch_cuda()
    ref, plan = _plan_pair(128, 8, 60, 400.0)
    O = ref.overlap
    sizes = [O // 3, O // 3, O // 2, 3000, 1, 4097, 2500, 777]
    total = sum(sizes)
    x = synth.uniform_u8(128, total, 21)
    st = tx.Stream(plan, max(sizes))
    outs = []
    pos = 0
    for k, n in enumerate(sizes):
        blk = torch.from_numpy(np.ascontiguousarray(x[:, pos:pos + n]))
        blk = blk.to("cuda") if k % 2 else blk.pin_memory()
        d_out = torch.full((plan.ndm, round_up(max(n, 2), 2)), -1, dtype=torch.int32, device="cuda")
        got = st.push(blk, n, d_out)
        torch.cuda.synchronize()
        outs.append(d_out[:, :got].cpu().numpy())
        pos += n
        _say(f"push {k}: {n} -> {got}")
    y = np.concatenate(outs, axis=1)
    assert y.shape[1] == total - O
    assert st.position() == (total, total - O)
    want = oracle.dedisperse_subband(x, ref, total - O)
    assert np.array_equal(y, want)


def test_stream_snapshot_restore_and_reset():
    torch = torch_cuda()
    ref, plan = _plan_pair(64, 8, 40, 300.0)
    O = ref.overlap
    n = 1500
    x = synth.uniform_u8(64, O + 6 * n, 22)
    a = tx.Stream(plan, n + O)
    d = torch.empty((plan.ndm, n), dtype=torch.int32, device="cuda")
    first = torch.empty((plan.ndm, round_up(O + n, 2)), dtype=torch.int32, device="cuda")
    assert a.push(torch.from_numpy(np.ascontiguousarray(x[:, :O + n])).to("cuda"), O + n, first) == n
    hist, held, rec, emi = a.snapshot()
    assert held == O and rec == O + n and emi == n
    b = tx.Stream(plan, n + O)
    b.restore(hist, held, rec, emi)
    for k in range(3):
        blk = torch.from_numpy(np.ascontiguousarray(x[:, O + n + k * n:O + n + (k + 1) * n])).to("cuda")
        da = torch.empty((plan.ndm, n), dtype=torch.int32, device="cuda")
        db = torch.empty((plan.ndm, n), dtype=torch.int32, device="cuda")
        assert a.push(blk, n, da) == n
        assert b.push(blk, n, db) == n
        torch.cuda.synchronize()
        assert torch.equal(da, db)
    want = oracle.dedisperse_subband(x[:, n + 2 * n:], ref, n)
    assert np.array_equal(db.cpu().numpy(), want)
    b.reset()
    assert b.position() == (0, 0)
    assert b.push(torch.from_numpy(np.ascontiguousarray(x[:, :n])).to("cuda"), n, d) == max(0, n - O)
    del d


BEAMS = [  # (nchan, nsub, ndm, dmmax, nt, f_top, f_bot, tsamp)
    (256, 16, 128, 508.0, 8192, 1712.0, 856.0, 306.24e-6),
    (64, 8, 40, 300.0, 3000, 1712.0, 856.0, 306.24e-6),
    (320, 32, 100, 1500.0, 5000, 1088.0, 544.0, 153.12e-6),
    (128, 4, 70, 200.0, 4100, 1500.0, 1100.0, 1e-3),
    (48, 48, 33, 900.0, 777, 1500.0, 1100.0, 5e-4),
    (1024, 64, 100, 1000.0, 3000, 1712.0, 856.0, 153.12e-6),   # g = 14: 16 trials per second-stage workgroup
]


def _beam_setup(k, spec, torch):
    nchan, nsub, ndm, dmmax, nt, ft, fb, ts = spec
    ref, plan = _plan_pair(nchan, nsub, ndm, dmmax, ft, fb, ts)
    x = synth.normal_u8(nchan, nt + ref.overlap, 100 + k)
    d_in = device_block(x)
    y = torch.full((ndm, round_up(nt, 2)), -1, dtype=torch.int32, device="cuda")
    peaks = (torch.empty(ndm, dtype=torch.float64, device="cuda"), torch.empty(ndm, dtype=torch.int32, device="cuda"),
             torch.empty(ndm, dtype=torch.int64, device="cuda"))
    cands = torch.zeros((1 << 16, 3), dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    return dict(ref=ref, plan=plan, x=x, d_in=d_in, y=y, peaks=peaks, cands=cands, count=count, nt=nt)


def _check_beam(b, widths, gamma):
    nt = b["nt"]
    want = oracle.dedisperse_subband(b["x"], b["ref"], nt)
    got = b["y"][:, :nt].cpu().numpy()
    assert np.array_equal(got, want)
    ws, ww, wt = oracle.boxcar_peaks(want, widths)
    assert np.array_equal(b["peaks"][0].cpu().numpy(), ws)
    assert np.array_equal(b["peaks"][1].cpu().numpy(), ww) and np.array_equal(b["peaks"][2].cpu().numpy(), wt)
    wc = oracle.boxcar_candidates(want, widths, gamma)
    n = int(b["count"].item())
    assert n == len(wc)
    assert as_tuples(tx.parse_candidates(b["cands"].cpu().numpy(), n)) == wc


@pytest.mark.parametrize("graph", [False, True])
def test_batch_of_uneven_beams_matches_oracle(graph):
    torch = torch_cuda()
    widths = [1, 2, 4, 8, 16, 32]
    gamma = 4.5
    beams = [_beam_setup(k, spec, torch) for k, spec in enumerate(BEAMS)]
    batch = tx.Batch(8, graph=graph)
    s = torch.cuda.Stream()
    for b in beams:
        batch.add(b["plan"], b["d_in"], b["nt"], b["y"], widths=widths, gamma=gamma, peaks=b["peaks"],
                  cands=b["cands"], count=b["count"])
    assert batch.done()                            # nothing launched yet
    batch.wait()
    with torch.cuda.stream(s):
        for rep in range(3):
            _say(f"batch launch graph={graph} rep={rep}")
            for b in beams:
                b["y"].fill_(-5)
                b["count"].fill_(-1)
            batch.launch(s)
            batch.wait()                           # the batch's own completion, not the stream's
            assert batch.done()
            for b in beams:
                _check_beam(b, widths, gamma)
            # new data for the next replay, written by eager work on the same stream
            for k, b in enumerate(beams):
                b["x"] = synth.normal_u8(b["x"].shape[0], b["x"].shape[1], 1000 * (rep + 1) + k)
                b["d_in"][:, :b["x"].shape[1]] = torch.from_numpy(b["x"]).to("cuda")
    # fewer jobs under the same batch (and graph)
    batch.clear()
    b = beams[1]
    batch.add(b["plan"], b["d_in"], b["nt"], b["y"], widths=widths, gamma=gamma, peaks=b["peaks"], cands=b["cands"],
              count=b["count"])
    with torch.cuda.stream(s):
        batch.launch(s)
        s.synchronize()
    _check_beam(b, widths, gamma)


def test_batch_result_same_alone_and_in_mix():
    torch = torch_cuda()
    widths = [1, 4, 16]
    beams = [_beam_setup(k, spec, torch) for k, spec in enumerate(BEAMS)]
    mix = tx.Batch(8)
    for b in beams:
        mix.add(b["plan"], b["d_in"], b["nt"], b["y"], widths=widths, gamma=5.0, peaks=b["peaks"], cands=b["cands"],
                count=b["count"])
    mix.launch()
    torch.cuda.synchronize()
    mixed = [(b["y"].clone(), [p.clone() for p in b["peaks"]], int(b["count"].item())) for b in beams]
    for k, b in enumerate(beams):
        alone = tx.Batch(1)
        b["y"].fill_(0)
        alone.add(b["plan"], b["d_in"], b["nt"], b["y"], widths=widths, gamma=5.0, peaks=b["peaks"],
                  cands=b["cands"], count=b["count"])
        alone.launch()
        torch.cuda.synchronize()
        nt = b["nt"]
        assert torch.equal(b["y"][:, :nt], mixed[k][0][:, :nt])
        for p, q in zip(b["peaks"], mixed[k][1]):
            assert torch.equal(p, q)
        assert int(b["count"].item()) == mixed[k][2]


@pytest.mark.parametrize("graph", [False, True])
def test_batch_of_streams_equals_single_streams(graph):
    torch = torch_cuda()
    specs = [(128, 8, 60, 400.0), (64, 4, 30, 250.0), (96, 12, 45, 600.0)]
    pairs = [_plan_pair(*sp) for sp in specs]
    block = 2000
    nblocks = 6
    xs = [synth.uniform_u8(sp[0], block * nblocks, 300 + k) for k, sp in enumerate(specs)]
    batched = [tx.Stream(p, block) for _, p in pairs]
    single = [tx.Stream(p, block) for _, p in pairs]
    batch = tx.Batch(4, graph=graph)
    s = torch.cuda.Stream()
    outs_b = [[] for _ in specs]
    outs_s = [[] for _ in specs]
    with torch.cuda.stream(s):
        for k in range(nblocks):
            _say(f"stream batch graph={graph} block {k}")
            batch.clear()
            blocks = [torch.from_numpy(np.ascontiguousarray(x[:, k * block:(k + 1) * block])).pin_memory() for x in xs]
            d_b = [torch.empty((p.ndm, block), dtype=torch.int32, device="cuda") for _, p in pairs]
            for q in range(len(specs)):
                batch.add_stream(batched[q], blocks[q], block, d_b[q])
            batch.launch(s)
            n_b = [batch.stream_output(q) for q in range(len(specs))]
            for q in range(len(specs)):
                d_s = torch.empty((pairs[q][1].ndm, block), dtype=torch.int32, device="cuda")
                n_s = single[q].push(blocks[q], block, d_s, stream=s)
                assert n_s == n_b[q]
                s.synchronize()
                outs_b[q].append(d_b[q][:, :n_b[q]].cpu().numpy())
                outs_s[q].append(d_s[:, :n_s].cpu().numpy())
    for q, (ref, _) in enumerate(pairs):
        yb = np.concatenate(outs_b[q], axis=1)
        ys = np.concatenate(outs_s[q], axis=1)
        assert np.array_equal(yb, ys)
        n = yb.shape[1]
        assert n == block * nblocks - ref.overlap
        assert np.array_equal(yb, oracle.dedisperse_subband(xs[q], ref, n))


# One beam of each (channels, sub-bands, g) class of the uneven 64-beam batch,
# at full shape: 1024 channels / 64 sub-bands / g = 14 (16 trials per
# second-stage workgroup), 2048 / 128 / 26 and 4096 / 128 / 26 (13 per
# workgroup).  Indices into synth.batched_beams().
BATCHED_SAMPLE = [9, 1, 6, 0]


def _sampled_rows(ref, wl):
    rows = {0, 1, ref.g - 1, ref.g, ref.g + 1, ref.ndm // 2, ref.ndm - 1}
    for spec in wl.pulses:
        i = int(np.argmin(np.abs(ref.dms - spec[1])))
        rows |= {max(i - 1, 0), i, min(i + 1, ref.ndm - 1)}
    return sorted(rows)


@pytest.mark.slow
def test_batched_beams_full_shape_sampled_rows():
    """Beams of the uneven batch at their real shapes (with their pulses), in
    one graph-replayed batch launch: sampled rows against the oracle's
    effective-offset sum, with the rows' peaks and candidates."""
    torch = torch_cuda()
    beams = synth.batched_beams()
    jobs = []
    for k in BATCHED_SAMPLE:
        wl = beams[k]
        plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, 0)
        ref = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms, plan.nsub)
        assert (ref.g, ref.overlap) == (plan.g, plan.overlap)
        _say(f"batched beam {k}: nchan={plan.nchan} nsub={plan.nsub} g={plan.g} ndm={plan.ndm} nt={wl.nt}")
        pulses = synth.place_pulses(wl, lambda dm: oracle.delay_samples(dm, wl.freqs, ref.fref, wl.tsamp))
        n = wl.nt + ref.overlap
        d_in = synth.device_normal_u8(torch, plan.nchan, round_up(n, 256), wl.seed, pulses=pulses)
        y = torch.full((plan.ndm, wl.nt), -3, dtype=torch.int32, device="cuda")
        peaks = (torch.empty(plan.ndm, dtype=torch.float64, device="cuda"),
                 torch.empty(plan.ndm, dtype=torch.int32, device="cuda"),
                 torch.empty(plan.ndm, dtype=torch.int64, device="cuda"))
        cands = torch.zeros((1 << 18, 3), dtype=torch.int64, device="cuda")
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
        jobs.append(dict(k=k, wl=wl, plan=plan, ref=ref, d_in=d_in, y=y, peaks=peaks, cands=cands, count=count))
    batch = tx.Batch(len(jobs), graph=True)
    for j in jobs:
        batch.add(j["plan"], j["d_in"], j["wl"].nt, j["y"], widths=j["wl"].widths, gamma=j["wl"].gamma,
                  peaks=j["peaks"], cands=j["cands"], count=j["count"])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(2):                      # capture, then a replay
            _say(f"batched beams launch {rep}")
            for j in jobs:
                j["y"].fill_(-3)
            batch.launch(s)
            s.synchronize()
    batch.close()
    for j in jobs:
        wl, ref = j["wl"], j["ref"]
        rows = _sampled_rows(ref, wl)
        _say(f"beam {j['k']}: oracle on rows {rows}")
        x = j["d_in"][:, :wl.nt + ref.overlap].cpu().numpy()
        want = oracle.dedisperse_offsets(x, ref.offsets[rows], wl.nt)
        assert np.array_equal(j["y"][rows].cpu().numpy(), want)
        ws, ww, wt = oracle.boxcar_peaks(want, wl.widths)
        p = [t.cpu().numpy() for t in j["peaks"]]
        assert np.array_equal(p[0][rows], ws)
        assert np.array_equal(p[1][rows], ww) and np.array_equal(p[2][rows], wt)
        n = int(j["count"].item())
        assert n < (1 << 18)
        wc = [(rows[d], t, w, v) for (d, t, w, v) in oracle.boxcar_candidates(want, wl.widths, wl.gamma)]
        got = [c for c in as_tuples(tx.parse_candidates(j["cands"].cpu().numpy(), n)) if c[0] in set(rows)]
        assert got == wc
        del x
