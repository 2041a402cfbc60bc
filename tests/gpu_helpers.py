"""Shared helpers for the GPU tests: move seeded inputs to the device, call
the HIP library through its binding, and bring results back."""

import numpy as np

import paper_2401_13834_amd as tx


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def round_up(v, m):
    return (v + m - 1) // m * m


def device_block(x, pitch=None):
    """uint8 device tensor [nchan, pitch] holding x (rows padded with zeros)."""
    torch = torch_cuda()
    nchan, n = x.shape
    pitch = pitch or round_up(max(n, 1), 256)
    d = torch.zeros((nchan, pitch), dtype=torch.uint8, device="cuda")
    d[:, :n] = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    return d


def gpu_dedisperse(plan, x, nt, out_pitch=None, fill=-7, ws=False, d_in=None):
    torch = torch_cuda()
    ndm = plan.ndm
    out_pitch = out_pitch or max(round_up(nt, 2), 2)
    if d_in is None:
        d_in = device_block(x)
    out = torch.full((ndm, out_pitch), fill, dtype=torch.int32, device="cuda")
    if ws:
        n = plan.ws_size(nt)
        wsb = torch.empty(max(n, 256), dtype=torch.uint8, device="cuda")
        tx.tx_dedisperse(plan, d_in, nt, out, ws=wsb)
    else:
        tx.tx_dedisperse(plan, d_in, nt, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_peaks(dmt_dev, nt, widths):
    torch = torch_cuda()
    ndm = dmt_dev.shape[0]
    snr = torch.empty(ndm, dtype=torch.float64, device="cuda")
    wid = torch.empty(ndm, dtype=torch.int32, device="cuda")
    tim = torch.empty(ndm, dtype=torch.int64, device="cuda")
    tx.tx_boxcar_snr(dmt_dev, nt, widths, snr, wid, tim)
    torch.cuda.synchronize()
    return snr.cpu().numpy(), wid.cpu().numpy(), tim.cpu().numpy()


def gpu_candidates(dmt_dev, nt, widths, gamma, cap=1 << 20, with_peaks=False):
    torch = torch_cuda()
    ndm = dmt_dev.shape[0]
    raw = torch.zeros((max(cap, 1), 3), dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    peaks = None
    if with_peaks:
        peaks = (torch.empty(ndm, dtype=torch.float64, device="cuda"),
                 torch.empty(ndm, dtype=torch.int32, device="cuda"),
                 torch.empty(ndm, dtype=torch.int64, device="cuda"))
    tx.tx_candidates(dmt_dev, nt, widths, gamma, raw[:cap] if cap else raw[:0], count, peaks=peaks)
    torch.cuda.synchronize()
    n = int(count.item())
    rec = tx.parse_candidates(raw.cpu().numpy(), min(n, cap))
    if with_peaks:
        return n, rec, tuple(t.cpu().numpy() for t in peaks)
    return n, rec


def as_tuples(rec):
    return [(int(r["dm_index"]), int(r["time"]), int(r["width"]), float(r["snr"])) for r in rec]
