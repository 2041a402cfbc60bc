"""DM-time clustering (Sec. 2.5): the HIP DBSCAN against the oracle's
dbscan_plane, point by point, and at sizes the oracle cannot reach against
scikit-learn's DBSCAN on the properties that define a clustering."""

import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2401_13834_amd as tx
from gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _records(raw):
    rec = np.ascontiguousarray(raw).view(np.uint8).reshape(-1).view(tx.CAND_DTYPE)
    return [(int(r["dm_index"]), int(r["time"]), int(r["width"]), float(r["snr"])) for r in rec]


def _plan(ndm, dm_step, nchan=64, tsamp=1e-3):
    freqs = synth.band_centres(1712.0, 856.0, nchan)
    dms = np.arange(ndm, dtype=np.float64) * dm_step
    return freqs, dms, tsamp, tx.tx_plan(freqs, tsamp, dms, 8)


def _gpu_cluster(torch, plan, raw, radius, min_pts):
    cands = torch.from_numpy(raw).to("cuda")
    srt, lab, rep, ncl = tx.tx_cluster(plan, cands, raw.shape[0], radius, min_pts)
    torch.cuda.synchronize()
    return _records(srt.cpu().numpy()), lab.cpu().numpy(), rep.cpu().numpy(), int(ncl.item())


@pytest.mark.parametrize("n,radius,min_pts,seed", [(300, 4.0, 2, 1), (1500, 8.0, 3, 2), (800, 16.0, 5, 3),
                                                   (600, 6.5, 0, 4), (1, 4.0, 0, 5), (2000, 2.0, 1, 6)])
def test_cluster_matches_oracle(n, radius, min_pts, seed):
    torch = torch_cuda()
    _say(f"cluster n={n} r={radius} k={min_pts}")
    freqs, dms, tsamp, plan = _plan(120, 0.3)
    raw = synth.plane_points(n, 120, 3000, seed, blob_size=60, spread=2)
    srt, lab, rep, ncl = _gpu_cluster(torch, plan, raw, radius, min_pts)
    pts = _records(raw)
    w_srt, w_lab, w_rep, w_ncl = oracle.dbscan_plane([(d, t, w, s) for d, t, w, s in pts], dms, freqs, tsamp,
                                                     radius, min_pts)
    assert srt == w_srt
    assert ncl == w_ncl
    assert np.array_equal(lab, w_lab)
    assert np.array_equal(rep[:ncl], w_rep)
    assert np.all(rep[ncl:] == -1)


def test_cluster_empty_and_foreign_points():
    torch = torch_cuda()
    freqs, dms, tsamp, plan = _plan(50, 1.0)
    empty = np.zeros((0, 3), dtype=np.int64)
    srt, lab, rep, ncl = _gpu_cluster(torch, plan, empty, 5.0, 1)
    assert ncl == 0 and len(lab) == 0
    # records outside the plan's trials are noise and disturb nothing else
    raw = synth.plane_points(200, 50, 1000, 9, blob_size=40, spread=2)
    bad = raw.copy()
    bad[:5, 0] = (bad[:5, 0] & ~0xFFFFFFFF) | 50          # dm_index = ndm
    srt, lab, rep, ncl = _gpu_cluster(torch, plan, bad, 5.0, 1)
    keep = [p for p in srt if p[0] < 50]
    w_srt, w_lab, w_rep, w_ncl = oracle.dbscan_plane(keep, dms, freqs, tsamp, 5.0, 1)
    assert srt[:len(keep)] == w_srt and ncl == w_ncl
    assert np.array_equal(lab[:len(keep)], w_lab) and np.all(lab[len(keep):] == -1)


def test_cluster_rejects_bad_arguments():
    torch = torch_cuda()
    freqs, dms, tsamp, plan = _plan(10, 1.0)
    raw = torch.zeros((4, 3), dtype=torch.int64, device="cuda")
    with pytest.raises(tx.TxError):
        tx.tx_cluster(plan, raw, 4, 0.0, 1)
    with pytest.raises(tx.TxError):
        tx.tx_cluster(plan, raw, 4, 3.0, -1)
    with pytest.raises(tx.TxError):
        tx.tx_cluster(plan, raw, -1, 3.0, 1)


def test_cluster_of_pipeline_candidates():
    # The plain-256 block through dedispersion and a low threshold, clustered:
    # the injected pulse's detections collapse to one cluster whose
    # representative sits at the pulse.
    torch = torch_cuda()
    wl = synth.workload("plain-256")
    plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    ref = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    amp, dm, t0, w = 96.0, 200.0, 4000, 4
    start = t0 + plan.delays(dm).astype(np.int64)
    x = synth.normal_u8(len(wl.freqs), wl.nt + ref.overlap, 7, pulses=[(start, w, amp)])
    from gpu_helpers import device_block
    d_in = device_block(x)
    y = torch.empty((plan.ndm, wl.nt), dtype=torch.int32, device="cuda")
    tx.tx_dedisperse(plan, d_in, wl.nt, y)
    cands = torch.zeros((1 << 16, 3), dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    tx.tx_candidates(y, wl.nt, wl.widths, 5.0, cands, count)
    torch.cuda.synchronize()
    n = int(count.item())
    assert 0 < n < (1 << 16)
    srt, lab, rep, ncl = tx.tx_cluster(plan, cands, n, 8.0, 3)
    torch.cuda.synchronize()
    srt_h = _records(srt.cpu().numpy())
    lab_h, rep_h, ncl_h = lab.cpu().numpy(), rep.cpu().numpy(), int(ncl.item())
    pts = _records(cands[:n].cpu().numpy())
    w_srt, w_lab, w_rep, w_ncl = oracle.dbscan_plane(pts, wl.dms, wl.freqs, wl.tsamp, 8.0, 3)
    assert srt_h == w_srt and ncl_h == w_ncl
    assert np.array_equal(lab_h, w_lab) and np.array_equal(rep_h[:ncl_h], w_rep)
    best = max(range(ncl_h), key=lambda c: srt_h[rep_h[c]][3])
    d, t, _, _ = srt_h[rep_h[best]]
    assert abs(wl.dms[d] - dm) <= 8.0 and abs(t - t0) <= 8


@pytest.mark.parametrize("n,radius", [(100000, 4.0), (100000, 16.0)])
def test_cluster_large_against_scikit_learn(n, radius):
    # At sizes past the oracle: the same core points, the same partition of
    # them (compared as the map from core point to its cluster's first core
    # point), the same noise, valid border assignments.
    from sklearn.cluster import DBSCAN
    torch = torch_cuda()
    min_pts = 4
    freqs, dms, tsamp, plan = _plan(2048, 0.5, nchan=256, tsamp=1.5312e-4)
    raw = synth.plane_points(n, 2048, 65536, 21)
    _say(f"cluster large n={n} r={radius}")
    srt, lab, rep, ncl = _gpu_cluster(torch, plan, raw, radius, min_pts)
    xs = oracle.delay_axis(dms, freqs, tsamp)
    X = np.array([[xs[d], t] for d, t, _, _ in srt], dtype=np.float64)
    assert all(srt[i][:2] < srt[i + 1][:2] for i in range(len(srt) - 1))
    sk = DBSCAN(eps=radius, min_samples=min_pts + 2, algorithm="kd_tree").fit(X)
    core = np.zeros(len(srt), dtype=bool)
    core[sk.core_sample_indices_] = True
    assert ncl == len(set(sk.labels_[core]))
    # partition of core points: first core index per label must map one to one
    first_us, first_sk = {}, {}
    for i in np.nonzero(core)[0]:
        first_us.setdefault(int(lab[i]), int(i))
        first_sk.setdefault(int(sk.labels_[i]), int(i))
    assert sorted(first_us.values()) == sorted(first_sk.values())
    m_us = np.array([first_us[int(lab[i])] for i in np.nonzero(core)[0]])
    m_sk = np.array([first_sk[int(sk.labels_[i])] for i in np.nonzero(core)[0]])
    assert np.array_equal(m_us, m_sk)
    assert np.array_equal(lab < 0, sk.labels_ < 0)
    # clusters numbered by first core point, representatives are cluster maxima
    order = sorted(first_us, key=lambda c: first_us[c])
    assert order == list(range(ncl))
    snr = np.array([p[3] for p in srt])
    best = np.full(ncl, -np.inf)
    np.maximum.at(best, lab[lab >= 0], snr[lab >= 0])
    assert np.array_equal(snr[rep[:ncl]], best)
