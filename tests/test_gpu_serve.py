"""The serving loop: beams of uneven shape stream consecutive blocks at
Poisson arrivals; each block's DM x time array, peaks and candidates must be
the same as when the beam runs alone, and equal to the oracle on the beam's
concatenated input."""

import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2401_13834_amd as tx
from paper_2401_13834_amd import serve
from gpu_helpers import as_tuples, round_up, torch_cuda

pytestmark = pytest.mark.gpu

SPECS = [(64, 8, 40, 300.0), (128, 8, 60, 400.0), (96, 12, 45, 600.0), (48, 4, 33, 900.0), (160, 16, 70, 250.0)]
BLOCK = 3000
NBLOCKS = 6
WIDTHS = [1, 2, 4, 8, 16, 32]
GAMMA = 3.5
CAP = 8192


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def beams():
    torch = torch_cuda()
    out = []
    for k, (nchan, nsub, ndm, dmmax) in enumerate(SPECS):
        freqs = synth.band_centres(1712.0, 856.0, nchan)
        dms = np.linspace(0.0, dmmax, ndm)
        ref = oracle.make_plan(freqs, 306.24e-6, dms, nsub)
        plan = tx.tx_plan(freqs, 306.24e-6, dms, nsub)
        x = synth.normal_u8(nchan, BLOCK * NBLOCKS, 700 + k)
        host = [torch.from_numpy(np.ascontiguousarray(x[:, j * BLOCK:(j + 1) * BLOCK])).pin_memory()
                for j in range(NBLOCKS)]
        dev = [h.to("cuda") for h in host]
        out.append(dict(ref=ref, plan=plan, x=x, host=host, dev=dev))
    return out


def _alone(b):
    """The beam pushed block by block through its own stream, then boxcar."""
    torch = torch_cuda()
    plan = b["plan"]
    st = tx.Stream(plan, BLOCK)
    res = []
    for j in range(NBLOCKS):
        d = torch.full((plan.ndm, round_up(BLOCK, 2)), -3, dtype=torch.int32, device="cuda")
        n = st.push(b["dev"][j], BLOCK, d)
        if n == 0:
            res.append((0, None, None, None))
            continue
        peaks = (torch.empty(plan.ndm, dtype=torch.float64, device="cuda"),
                 torch.empty(plan.ndm, dtype=torch.int32, device="cuda"),
                 torch.empty(plan.ndm, dtype=torch.int64, device="cuda"))
        raw = torch.zeros((CAP, 3), dtype=torch.int64, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        tx.tx_candidates(d, n, WIDTHS, GAMMA, raw, cnt, peaks=peaks)
        torch.cuda.synchronize()
        c = int(cnt.item())
        res.append((n, d[:, :n].cpu().numpy(), [p.cpu().numpy() for p in peaks],
                    tx.parse_candidates(raw.cpu().numpy(), c)))
    st.close()
    return res


@pytest.mark.parametrize("graph,source,lanes,slots,budget", [
    (True, "host", 2, 3, None),
    (False, "device", 1, 5, None),
    (True, "device", 3, 2, None),
    (True, "host", 2, 8, "one-slot"),
])
def test_served_blocks_same_alone_and_in_mix(beams, graph, source, lanes, slots, budget):
    torch = torch_cuda()
    plans = [b["plan"] for b in beams]
    mem = None
    if budget == "one-slot":
        probe = serve.Server(plans, BLOCK, WIDTHS, gamma=GAMMA, cap=CAP, lanes=lanes, max_slots=1, mem_budget=1 << 40,
                             graph=graph, source=source)
        mem = probe.per_slot_bytes * lanes + 1
        probe.close()
    srv = serve.Server(plans, BLOCK, WIDTHS, gamma=GAMMA, cap=CAP, lanes=lanes, max_slots=slots, mem_budget=mem,
                       graph=graph, source=source, keep=("peaks", "cands", "dmt"))
    if budget == "one-slot":
        assert srv.slots == 1
    arrivals = synth.poisson_arrivals(len(beams), NBLOCKS, 0.02, 4.0, 31)
    key = "host" if source == "host" else "dev"

    def data(b, j):
        return beams[b][key][j]

    _say(f"serve graph={graph} source={source} lanes={lanes} slots={srv.slots}")
    results, stats = srv.run(arrivals, data)
    srv.close()
    _say(f"served {stats.blocks} blocks in {stats.batches} batches (mean {stats.mean_batch:.2f}), "
         f"p50 {stats.p50_s * 1e3:.2f} ms p99 {stats.p99_s * 1e3:.2f} ms")
    assert stats.blocks == len(beams) * NBLOCKS
    assert len(results) == stats.blocks
    if srv.slots > 1:
        assert stats.mean_batch > 1.0          # blocks of different beams shared launches
    assert all(r.latency >= 0 for r in results)
    by_beam = {}
    for r in results:
        by_beam.setdefault(r.beam, []).append(r)
    for bi, b in enumerate(beams):
        rs = by_beam[bi]
        assert [r.index for r in rs] == list(range(NBLOCKS))
        alone = _alone(b)
        ref = b["ref"]
        O = ref.overlap
        outs = []
        for r, (n, dmt, peaks, cands) in zip(rs, alone):
            assert r.n_out == n
            if n == 0:
                continue
            assert np.array_equal(r.dmt, dmt)
            assert np.array_equal(r.snr, peaks[0]) and np.array_equal(r.width, peaks[1])
            assert np.array_equal(r.time, peaks[2])
            assert r.count == len(cands)
            assert as_tuples(r.cands) == as_tuples(cands)
            outs.append(r.dmt)
        y = np.concatenate(outs, axis=1)
        total = BLOCK * NBLOCKS
        assert y.shape[1] == total - O
        want = oracle.dedisperse_subband(b["x"], ref, total - O)
        assert np.array_equal(y, want)
        # one emitted block's boxcar against the oracle
        last = rs[-1]
        blk = want[:, -last.n_out:]
        ws, ww, wt = oracle.boxcar_peaks(blk, WIDTHS)
        assert np.array_equal(last.snr, ws) and np.array_equal(last.width, ww) and np.array_equal(last.time, wt)
        assert as_tuples(last.cands) == oracle.boxcar_candidates(blk, WIDTHS, GAMMA)


OCT_BLOCKS = 7          # 343278 samples of history prime the first 5.2 blocks


@pytest.mark.slow
def test_octave_beams_served_alone_and_oracle():
    """Two multi-octave beams (8192 channels over 544-1088 MHz, 8192 trials
    to DM 5000, 65536-sample blocks, widths to 1024) served at Poisson
    arrivals on two lanes: every block's sampled rows, peaks and candidates
    equal the beam pushed alone through its own stream, and the sampled rows
    of the concatenated output equal the oracle (the C oracle on the coarse
    groups that hold them)."""
    from oracle import c_oracle as co
    torch = torch_cuda()
    wl = synth.workload("octave-8192")
    plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    nchan, nt, g = plan.nchan, wl.nt, plan.g
    groups = [0, 4095 // g, plan.ngroups - 2]                     # low DM, near DM 2500, high DM
    rows = sorted(j * g + i for j in groups for i in (0, g // 2, g - 1))
    beams = []
    for k in range(2):
        d = synth.device_normal_u8(torch, nchan, nt * OCT_BLOCKS, 900 + k)
        beams.append([d[:, j * nt:(j + 1) * nt] for j in range(OCT_BLOCKS)])
    srv = serve.Server([plan, plan], nt, wl.widths, gamma=wl.gamma, cap=1 << 16, lanes=2, max_slots=2, graph=True,
                       source="device", keep=("peaks", "cands", "dmt"), dmt_rows=rows)
    arrivals = synth.poisson_arrivals(2, OCT_BLOCKS, 0.05, 2.0, 57)
    _say(f"octave serve: slots {srv.slots}, rows {rows}")
    results, stats = srv.run(arrivals, lambda b, j: beams[b][j])
    srv.close()
    assert stats.blocks == 2 * OCT_BLOCKS
    by_beam = {}
    for r in results:
        by_beam.setdefault(r.beam, []).append(r)
    for b in range(2):
        rs = by_beam[b]
        st = tx.Stream(plan, nt)
        outs = []
        for j, r in enumerate(rs):
            d = torch.empty((plan.ndm, nt), dtype=torch.int32, device="cuda")
            n = st.push(beams[b][j], nt, d)
            assert r.n_out == n
            if n == 0:
                continue
            peaks = (torch.empty(plan.ndm, dtype=torch.float64, device="cuda"),
                     torch.empty(plan.ndm, dtype=torch.int32, device="cuda"),
                     torch.empty(plan.ndm, dtype=torch.int64, device="cuda"))
            raw = torch.zeros((1 << 16, 3), dtype=torch.int64, device="cuda")
            cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
            tx.tx_candidates(d[:, :n], n, wl.widths, wl.gamma, raw, cnt, peaks=peaks)
            torch.cuda.synchronize()
            assert np.array_equal(r.dmt, d[rows, :n].cpu().numpy())
            assert np.array_equal(r.snr, peaks[0].cpu().numpy()) and np.array_equal(r.width, peaks[1].cpu().numpy())
            assert np.array_equal(r.time, peaks[2].cpu().numpy())
            c = int(cnt.item())
            assert r.count == c
            assert as_tuples(r.cands) == as_tuples(tx.parse_candidates(raw.cpu().numpy(), c))
            outs.append(r.dmt)
            del d, raw
        st.close()
        y = np.concatenate(outs, axis=1)
        total = nt * OCT_BLOCKS - plan.overlap
        assert y.shape[1] == total
        _say(f"octave beam {b}: C oracle on groups {groups}")
        x = torch.cat(beams[b], dim=1).cpu().numpy()
        for jg in groups:
            want = co.dedisperse_subband(x, wl.freqs, wl.tsamp, wl.dms[jg * g:(jg + 1) * g], wl.nsub, g, total)
            for i in range(g):
                row = jg * g + i
                if row in rows:
                    assert np.array_equal(y[rows.index(row)], want[i]), row
        del x
    torch.cuda.empty_cache()
