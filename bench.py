#!/usr/bin/env python3
"""Throughput benchmark of the dedispersion + matched-filter hot path.

One step = two-stage sub-band dedispersion of one resident uint8 block
(tx_dedisperse) followed by the boxcar matched filter with per-DM peaks and
the thresholded candidate list (tx_candidates), all on one GPU through the C
ABI.  Prints one JSON line.

Default workload ``paper-4096``: 4096 channels over 856-1712 MHz, 153.12 us,
65536-sample blocks, 4096 DM trials 0..2047.5, 64 sub-bands, widths 1..512,
seeded synthetic noise with ten dispersed pulses.
"""

from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ADD16 = 256 * 4 * 16 * 2 * 2.4e9   # 16-bit integer adds/s: 256 CUs x 64 lanes x 2 (packed) x 2.4 GHz
# Three-operand (VOP3) instructions per clock per CU measured by tx_peaks on
# MI355X (v_add3_u32 59.5, v_alignbyte_b32 58.7, v_perm_b32 59.8), and the
# bytes per clock per CU of the first stage's paired 4-byte LDS reads at its
# 9-dword lane stride (4.12 clocks per wavefront read of 512 bytes).
MEASURED_VOP3_PER_CLK_CU = 59.3
MEASURED_PAIRED_LDS_B_PER_CLK_CU = 124.3
PAPER_DM_SAMPLES_PER_S = 4096 / 153e-6  # real time on one CPU core, 4096 channels and trials, 153 us
# HBM rates that tx_peaks measures on this part, the practical ceilings beside
# the 8 TB/s published peak: a copy with 8 loads in flight per thread (bytes
# read + written per second) and a read-only stream.  The write rate follows
# from the two: a copy of B bytes takes B / read + B / write.
MEASURED_COPY_BYTES_PER_S = 4.91e12
MEASURED_READ_BYTES_PER_S = 5.94e12
MEASURED_WRITE_BYTES_PER_S = 1.0 / (2.0 / MEASURED_COPY_BYTES_PER_S - 1.0 / MEASURED_READ_BYTES_PER_S)


KERNEL_SOURCES = {"stage1": ("tx_kernels_dedisp.hip",), "stage2": ("tx_kernels_dedisp.hip",),
                  "boxcar": ("tx_kernels_boxcar.hip",), "transpose": ("tx_kernels_transpose.hip",),
                  "stats": ("tx_kernels_stats.hip",), "downsample2": ("tx_kernels_downsample.hip",),
                  "downsample4": ("tx_kernels_downsample.hip",),
                  # the batch launch: its persistent dedispersion and boxcar kernels,
                  # and the plan code that picks each beam's sub-band count
                  "batch": ("tx_kernels_dedisp.hip", "tx_kernels_boxcar.hip", "tx_plan.cpp")}


def kernel_source_hash(kernel):
    """Hash of the kernel's source files without comments and blank lines,
    so that the stored counters stay valid across edits of comments only."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2401_13834_amd", "csrc", name)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("\n".join(line.rstrip() for line in src.splitlines() if line.strip()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload, split=False):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (with split: bytes read and bytes
    written)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    ent = data.get(f"{kernel}:{workload}")
    if not ent or ent.get("source_hash") != kernel_source_hash(kernel):
        return None
    if split:
        if ent.get("read_bytes") is None or ent.get("write_bytes") is None:
            return None
        return ent["read_bytes"], ent["write_bytes"]
    return ent.get("hbm_bytes_per_launch")


def make_input(torch, plan, wl, synth, pitch):
    """Seeded noise with the workload's pulses, drawn on the device: every
    channel an independent N(128, 16^2) row, clipped and rounded to uint8."""
    return synth.device_normal_u8(torch, len(wl.freqs), pitch, wl.seed, pulses=place_pulses(plan, wl, synth))


def cpu_baseline(wl, x, g, seconds):
    """The C oracle (OpenMP over the host's cores), as it is, on a bounded
    sample of the same block: the first K coarse groups (K*g DM trials) over
    the full block length, through dedispersion, peaks and candidates.  The
    NumPy oracle's single-threaded rate on one group is reported beside it."""
    import oracle
    from oracle import c_oracle as co
    nt = wl.nt
    threads = co.max_threads()

    def run(k):
        t = time.perf_counter()
        y = co.dedisperse_subband(x, wl.freqs, wl.tsamp, wl.dms[:k * g], wl.nsub, g, nt, threads=threads)
        co.boxcar_peaks(y, wl.widths, threads=threads)
        co.boxcar_candidates(y, wl.widths, wl.gamma, threads=threads)
        return time.perf_counter() - t, k * g

    run(1)                                         # warm-up (builds the library if needed)
    dt1, _ = run(1)
    k = max(1, min(len(wl.dms) // g, int(seconds / max(dt1, 1e-3))))
    dt, ntrials = run(k)
    kmax = len(wl.dms) // g
    if dt < 0.5 * seconds and k < kmax:           # fixed costs made the first estimate short
        k = max(k + 1, min(kmax, int(k * seconds / max(dt, 1e-3))))
        dt, ntrials = run(k)
    reps = 1
    if dt < 0.5 * seconds:                        # the whole block is quick: repeat it
        reps = max(1, int(seconds / max(dt, 1e-3)))
        total, n = 0.0, 0
        for _ in range(reps):
            d1, n1 = run(k)
            total += d1
            n += n1
        dt, ntrials = total, n
    ref = oracle.make_plan(wl.freqs, wl.tsamp, wl.dms[:g], wl.nsub, g=g)
    t = time.perf_counter()
    yn = oracle.dedisperse_subband(x[:, :nt + ref.overlap], ref, nt)
    oracle.boxcar_peaks(yn, wl.widths)
    oracle.boxcar_candidates(yn, wl.widths, wl.gamma)
    dtn = time.perf_counter() - t
    return {"value": ntrials * nt / dt, "unit": "DM-trial samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{ntrials // reps} of {len(wl.dms)} DM trials ({k} coarse groups of {g}) x {nt} samples"
                      f"{f', run {reps} times' if reps > 1 else ''}, "
                      f"two-stage dedispersion + peaks + candidates, C oracle with {threads} OpenMP threads, "
                      f"{dt:.1f} s",
            "numpy_oracle_1core": g * nt / dtn}


def place_pulses(plan, wl, synth):
    """(start[nchan], width, amplitude) of the workload's pulses, placed with
    the plan's own brute-force delays."""
    return synth.place_pulses(wl, plan.delays)


def transpose_leg(torch, tx, nchan, nt, overlap, launches=20):
    """Time-major ingest: one recorded block (nt rows of nchan channel bytes)
    transposed into the channel rows of a stream buffer, at the position a
    block lands (after the overlap), timed per launch with HIP events.  Pure
    data movement: bytes = read + write of the block, against HBM peak."""
    gen = torch.Generator(device="cuda").manual_seed(11)
    d_tf = torch.randint(0, 256, (nt, nchan), dtype=torch.uint8, device="cuda", generator=gen)
    off = (overlap + 127) // 128 * 128
    pitch = (off + nt + 255) // 256 * 256
    ring = torch.empty((nchan, pitch), dtype=torch.uint8, device="cuda")
    dst = ring[:, off:]
    for _ in range(3):
        tx.tx_transpose_tf(d_tf, nchan, nt, dst)
    torch.cuda.synchronize()
    tx.tx_profile_collect(tx.TX_KERNEL_TRANSPOSE)
    tx.tx_profile_enable(True)
    for _ in range(launches):
        tx.tx_transpose_tf(d_tf, nchan, nt, dst)
    torch.cuda.synchronize()
    tx.tx_profile_enable(False)
    ms, n = tx.tx_profile_collect(tx.TX_KERNEL_TRANSPOSE)
    avg = ms / max(n, 1)
    ok = bool(torch.equal(ring[:, off:off + nt], d_tf.t()))
    nbytes = 2 * nchan * nt
    del d_tf, ring
    torch.cuda.empty_cache()
    return {"workload": f"one block as recorded, {nt} samples x {nchan} channels (uint8, time-major), "
                        f"into channel rows behind a {overlap}-sample history",
            "bytes_per_launch": nbytes, "avg_ms": avg, "launches": n,
            "achieved_GBps": nbytes / (avg * 1e-3) / 1e9, "peak_GBps": 8000.0,
            "frac": nbytes / (avg * 1e-3) / 8e12, "matches_torch_transpose": ok,
            "traffic": load_traffic("transpose", "paper-4096")}


def ranges_leg(torch, tx, synth, steps=10):
    """The paper-scale block in three DM ranges, coarser in DM and time as DM
    grows (synth.dm_ranges("ranges-4096")): downsampling and dedispersion of
    every range in one call, then peaks and candidates per range, against the
    block's real-time budget."""
    wl = synth.workload("paper-4096")
    ranges = synth.dm_ranges("ranges-4096")
    plans = [tx.tx_plan(wl.freqs, wl.tsamp * k, dms, wl.nsub) for dms, k in ranges]
    rg = tx.Ranges(plans, [k for _, k in ranges])
    nt = wl.nt
    nchan = len(wl.freqs)
    need = rg.input_len(nt)
    pitch = (need + 255) // 256 * 256
    d_in = synth.device_normal_u8(torch, nchan, pitch, wl.seed)
    outs = [torch.empty((p.ndm, nt // k), dtype=torch.int32, device="cuda") for p, (_, k) in zip(plans, ranges)]
    cap = 1 << 20
    cands = [torch.empty((cap, 3), dtype=torch.int64, device="cuda") for _ in ranges]
    counts = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in ranges]
    stream = torch.cuda.current_stream()

    def step():
        rg.dedisperse(d_in, nt, outs, stream=stream)
        for r, (_, k) in enumerate(ranges):
            tx.tx_candidates(outs[r], nt // k, wl.widths, wl.gamma, cands[r], counts[r], stream=stream)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    tx.tx_profile_collect(tx.TX_KERNEL_DOWNSAMPLE)
    tx.tx_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    tx.tx_profile_enable(False)
    ds_ms, ds_n = tx.tx_profile_collect(tx.TX_KERNEL_DOWNSAMPLE)
    # Downsampling moves (k + 1) bytes per output sample of each distinct factor.
    ds_bytes = 0
    for k in sorted(set(k for _, k in ranges if k > 1)):
        n_k = max(nt // k + p.overlap for p, (_, kk) in zip(plans, ranges) if kk == k)
        ds_bytes += nchan * n_k * (k + 1)
    ds_per_block = ds_ms / steps
    samples = sum(p.ndm * (nt // k) for p, (_, k) in zip(plans, ranges))
    out = {"workload": "ranges-4096", "ranges": [{"dm": [float(d[0]), float(d[-1])], "trials": len(d), "factor": k}
                                                 for d, k in ranges],
           "ms_per_block": dt * 1e3, "block_duration_ms": nt * wl.tsamp * 1e3,
           "dm_trial_samples_per_s": samples / dt, "unit": "DM-trial samples/s (at each range's sampling)",
           "candidates_last_step": [int(c.item()) for c in counts],
           "downsample": {"ms_per_block": ds_per_block, "launches_per_block": ds_n / steps,
                          "bytes_per_block": ds_bytes, "achieved_GBps": ds_bytes / (ds_per_block * 1e-3) / 1e9,
                          "peak_GBps": 8000.0, "frac": ds_bytes / (ds_per_block * 1e-3) / 8e12,
                          "traffic": [load_traffic("downsample2", "ranges-4096"),
                                      load_traffic("downsample4", "ranges-4096")]}}
    rg.close()
    del d_in, outs, cands
    torch.cuda.empty_cache()
    return out


def stats_leg(torch, tx, nchan, nt, launches=20):
    """Per-channel power sums (the statistics of the narrow-band RFI mask) of
    one paper-scale block: a pure read of the block, against HBM peak."""
    gen = torch.Generator(device="cuda").manual_seed(13)
    pitch = (nt + 255) // 256 * 256
    d_in = torch.randint(0, 256, (nchan, pitch), dtype=torch.uint8, device="cuda", generator=gen)
    sums = torch.empty((nchan, 4), dtype=torch.int64, device="cuda")
    for _ in range(3):
        tx.tx_channel_power_sums(d_in, nchan, nt, sums)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(launches):
        tx.tx_channel_power_sums(d_in, nchan, nt, sums)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / launches
    nbytes = nchan * nt
    del d_in
    torch.cuda.empty_cache()
    return {"workload": f"{nchan} channels x {nt} samples (uint8)", "bytes_per_launch": nbytes, "avg_ms": ms,
            "achieved_GBps": nbytes / (ms * 1e-3) / 1e9, "peak_GBps": 8000.0, "frac": nbytes / (ms * 1e-3) / 8e12,
            "traffic": load_traffic("stats", "paper-4096")}


def cluster_leg(torch, tx, synth, sizes=(1000, 10000, 100000, 1000000), radii=(4.0, 8.0, 16.0), min_pts=5,
                reps=5):
    """DBSCAN of the DM-time plane (the paper's clustering benchmark axes:
    time against the number of points, for radii of 4, 8 and 16 samples):
    seeded planes of blobs plus scattered points over the paper-4096 trial
    grid, one tx_cluster call each (it returns when its work is done)."""
    wl = synth.workload("paper-4096")
    plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    rows = []
    for n in sizes:
        raw = torch.from_numpy(synth.plane_points(n, plan.ndm, wl.nt, 31)).to("cuda")
        for r in radii:
            tx.tx_cluster(plan, raw, n, r, min_pts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                _, _, _, ncl = tx.tx_cluster(plan, raw, n, r, min_pts)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            rows.append({"points": n, "radius": r, "ms": dt * 1e3, "clusters": int(ncl.item()),
                         "points_per_s": n / dt})
        del raw
    return {"workload": "plane points over the paper-4096 trials (70% in blobs of 200)", "min_pts": min_pts,
            "runs": rows}


def plan_adds(plan, nt):
    """Additions of one block: N_c * N_f * T (first stage) + N_DM * nsub * T (second)."""
    return plan.ngroups * plan.nchan * nt + plan.ndm * plan.nsub * nt


def plan_alg_bytes(plan, nt):
    """Algorithmic HBM bytes of one block through dedispersion and the boxcar:
    the input read once (N_f (T + O) bytes), the DM x time array written once
    and read once by the boxcar (2 * 4 N_DM T)."""
    return plan.nchan * (nt + plan.overlap) + 8 * plan.ndm * nt


def tuned_classes(tx, tune, beams, effort, path):
    """Per (channels, DM range) class of the uneven batch: the sub-band count
    and tiles tune.plan_autotuned picks on the class's largest DM grid at
    16384 samples; every beam of the class then uses them."""
    classes = {}
    for wl in beams:
        key = (len(wl.freqs), float(wl.dms[-1]))
        if key not in classes or len(wl.dms) > len(classes[key].dms):
            classes[key] = wl
    out = {}
    for key, wl in sorted(classes.items()):
        plan, times = tune.plan_autotuned(wl.freqs, wl.tsamp, wl.dms, 16384, effort=effort, path=path)
        out[key] = (plan.nsub, plan.get_tiles(), times)
    return out


def batched_leg(torch, tx, synth, steps, tune_effort=0, tune=True):
    """64 beams of uneven shape (channels 1024-4096, blocks 16384-65536, 512-4096
    DM trials up to DM 3000) dedispersed with peaks and candidates in one batch
    launch (persistent kernels) replayed as a HIP graph; against the same jobs
    run one beam per launch, whose outputs the batch's must equal.  Run twice:
    with each plan's own sub-band count and default tiles, and with the
    sub-band count and tiles autotuned per (channels, DM range) class."""
    import tempfile
    from paper_2401_13834_amd import tune as tune_mod
    beams = synth.batched_beams()
    inputs = []
    for wl in beams:
        plan0 = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, 0)
        nchan, nt = len(wl.freqs), wl.nt
        pitch = (nt + plan0.overlap + 255) // 256 * 256
        # the largest overlap over the sub-band counts tried is below DM_max's brute-force reach + 16
        pitch = max(pitch, (nt + plan0.brute_reach + 512 + 255) // 256 * 256)
        d_in = synth.device_normal_u8(torch, nchan, pitch, wl.seed, pulses=place_pulses(plan0, wl, synth))
        inputs.append(d_in)
    stream = torch.cuda.Stream()
    t_tune = time.perf_counter()
    classes = {}
    if tune:
        with tempfile.TemporaryDirectory() as tmp:
            with torch.cuda.stream(stream):
                classes = tuned_classes(tx, tune_mod, beams, tune_effort, os.path.join(tmp, "tiles.json"))
    t_tune = time.perf_counter() - t_tune

    def run(tuned):
        jobs = []
        for wl, d_in in zip(beams, inputs):
            if tuned:
                nsub, tiles, _ = classes[(len(wl.freqs), float(wl.dms[-1]))]
                plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, nsub)
                plan.set_tiles(*tiles)
            else:
                plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, 0)
            ndm, nt = plan.ndm, wl.nt
            assert d_in.shape[1] >= nt + plan.overlap
            mk = lambda: dict(y=torch.empty((ndm, nt), dtype=torch.int32, device="cuda"),
                              peaks=(torch.empty(ndm, dtype=torch.float64, device="cuda"),
                                     torch.empty(ndm, dtype=torch.int32, device="cuda"),
                                     torch.empty(ndm, dtype=torch.int64, device="cuda")),
                              cands=torch.empty((1 << 16, 3), dtype=torch.int64, device="cuda"),
                              count=torch.zeros(1, dtype=torch.int64, device="cuda"))
            jobs.append(dict(wl=wl, plan=plan, d_in=d_in, b=mk(), p=mk()))
        batch = tx.Batch(len(jobs), graph=True)
        for j in jobs:
            o = j["b"]
            batch.add(j["plan"], j["d_in"], j["wl"].nt, o["y"], widths=j["wl"].widths, gamma=j["wl"].gamma,
                      peaks=o["peaks"], cands=o["cands"], count=o["count"])
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            batch.launch(stream)                   # captures the graph
            batch.wait()
            ev0.record(stream)
            for _ in range(steps):
                batch.launch(stream)
            ev1.record(stream)
            batch.wait()
            ev1.synchronize()                      # recorded after the batch's own completion event
            t_batch = ev0.elapsed_time(ev1) * 1e-3 / steps

            def plain_round():
                for j in jobs:
                    o = j["p"]
                    tx.tx_dedisperse(j["plan"], j["d_in"], j["wl"].nt, o["y"], stream=stream)
                    tx.tx_candidates(o["y"], j["wl"].nt, j["wl"].widths, j["wl"].gamma, o["cands"], o["count"],
                                     peaks=o["peaks"], stream=stream)
            plain_round()
            stream.synchronize()
            ev0.record(stream)
            plain_round()
            ev1.record(stream)
            stream.synchronize()
            t_plain = ev0.elapsed_time(ev1) * 1e-3
            # per-kernel times of one direct (not captured) launch of the same batch
            direct = tx.Batch(len(jobs), graph=False)
            for j in jobs:
                o = j["b"]
                direct.add(j["plan"], j["d_in"], j["wl"].nt, o["y"], widths=j["wl"].widths, gamma=j["wl"].gamma,
                           peaks=o["peaks"], cands=o["cands"], count=o["count"])
            direct.launch(stream)
            direct.wait()
            for k in (tx.TX_KERNEL_STAGE1, tx.TX_KERNEL_STAGE2, tx.TX_KERNEL_BOXCAR):
                tx.tx_profile_collect(k)
            tx.tx_profile_enable(True)
            direct.launch(stream)
            direct.wait()
            tx.tx_profile_enable(False)
            kern = {}
            for name, k in (("stage1", tx.TX_KERNEL_STAGE1), ("stage2", tx.TX_KERNEL_STAGE2),
                            ("boxcar", tx.TX_KERNEL_BOXCAR)):
                ms, n = tx.tx_profile_collect(k)
                kern[name] = {"ms": ms, "launches": n}
            direct.close()
        same = all(torch.equal(j["b"]["y"], j["p"]["y"]) and
                   all(torch.equal(a, b) for a, b in zip(j["b"]["peaks"], j["p"]["peaks"])) and
                   int(j["b"]["count"].item()) == int(j["p"]["count"].item()) for j in jobs)
        dm_samples = sum(j["plan"].ndm * j["wl"].nt for j in jobs)
        adds = sum(plan_adds(j["plan"], j["wl"].nt) for j in jobs)
        alg = sum(plan_alg_bytes(j["plan"], j["wl"].nt) for j in jobs)
        ncand = sum(int(j["b"]["count"].item()) for j in jobs)
        nsubs = {}
        for j in jobs:
            nsubs[str(j["plan"].nsub)] = nsubs.get(str(j["plan"].nsub), 0) + 1
        batch.close()
        del jobs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        tx.tx_pool_trim()
        return {"value": dm_samples / t_batch, "ms_per_launch": t_batch * 1e3, "launches": steps,
                "plain_value": dm_samples / t_plain, "plain_ms": t_plain * 1e3,
                "speedup_vs_plain": t_plain / t_batch, "same_as_plain": bool(same),
                "dm_samples_per_launch": dm_samples, "nsub_chosen": nsubs, "candidates": ncand,
                "kernels_ms_direct_launch": kern,
                "roofline": dict({"bound": "alu", "achieved": round(adds / t_batch / 1e12, 3),
                                  "peak": round(PEAK_ADD16 / 1e12, 3), "unit": "Tadd/s",
                                  "frac": round(adds / t_batch / PEAK_ADD16, 4), "adds_per_launch": adds,
                                  "alg_hbm_bytes_per_launch": alg, "alg_hbm_GBps": round(alg / t_batch / 1e9, 1),
                                  "alg_hbm_frac": round(alg / t_batch / 8e12, 4)},
                                 # counter bytes per launch, taken on the plan-default batch
                                 **({} if tuned or traffic is None else
                                    {"traffic": traffic, "traffic_over_alg": round(traffic / alg, 3),
                                     "hbm_GBps": round(traffic / t_batch / 1e9, 1),
                                     "hbm_frac": round(traffic / t_batch / 8e12, 4)}))}

    traffic = load_traffic("batch", "batched-64")
    plain_plans = run(False)
    print(f"batched (plan defaults): {json.dumps(plain_plans)}", file=sys.stderr, flush=True)
    out = {"workload": "batched-64", "beams": len(beams), "graph": True, "persistent": True}
    out.update(plain_plans)
    if tune:
        tuned = run(True)
        print(f"batched (autotuned): {json.dumps(tuned)}", file=sys.stderr, flush=True)
        out["autotuned"] = dict(tuned, classes={f"{k[0]}ch-dm{int(k[1])}": {"nsub": v[0], "tiles": list(v[1]),
                                                                             "ms_by_nsub": v[2]}
                                                for k, v in classes.items()},
                                tune_seconds=round(t_tune, 1),
                                gain_vs_plan_defaults=tuned["value"] / plain_plans["value"])
    del inputs
    torch.cuda.empty_cache()
    return out


def served_leg(torch, tx, synth, serve, runs_spec, lanes, max_slots):
    """256 beams stream consecutive 4096-channel, 32768-sample blocks at
    Poisson arrivals (mean gap = block duration / speed) through the
    continuous-batching loop; p50/p99 latency from arrival to host-visible
    candidates.  Source "host": blocks arrive in pinned host memory and the
    rate includes their PCIe upload; "device": blocks are already in HBM."""
    wl = synth.workload("served-4096")
    plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    nchan, nt = len(wl.freqs), wl.nt
    t_blk = nt * wl.tsamp
    adds_per_dm_sample = plan_adds(plan, nt) / (plan.ndm * nt)
    nbeams = 256
    runs = []
    slots = {}
    for source in ("host", "device"):
        mine = [(sp, nb) for (src, sp, nb) in runs_spec if src == source]
        if not mine:
            continue
        pool = []
        for i in range(4):
            d = synth.device_normal_u8(torch, nchan, nt, 4000 + i)
            pool.append(d if source == "device" else d.cpu().pin_memory())
        srv = serve.Server([plan] * nbeams, nt, wl.widths, gamma=wl.gamma, cap=4096, lanes=lanes,
                           max_slots=max_slots, graph=True, source=source, keep=())
        slots[source] = srv.slots

        def data(b, k):
            return pool[(b * 7 + k) % len(pool)]

        for speed, nblocks in mine:
            for st in srv.streams:
                st.reset()
            arr = synth.poisson_arrivals(nbeams, nblocks, t_blk, speed, 4 + speed)
            _, stats = srv.run(arr, data)
            runs.append({"source": source, "speed": speed, "blocks": stats.blocks, "batches": stats.batches,
                         "mean_batch": round(stats.mean_batch, 2), "p50_ms": stats.p50_s * 1e3,
                         "p99_ms": stats.p99_s * 1e3, "max_ms": stats.max_s * 1e3, "value": stats.throughput,
                         "gpu_busy": stats.gpu_s / stats.wall_s if stats.wall_s > 0 else None,
                         "lane_overlap": stats.lane_s / stats.gpu_s if stats.gpu_s > 0 else None,
                         "adds_per_s": stats.throughput * adds_per_dm_sample,
                         "frac_of_add_peak": stats.throughput * adds_per_dm_sample / PEAK_ADD16,
                         "p99_below_block": stats.p99_s < t_blk})
            print(f"served: {json.dumps(runs[-1])}", file=sys.stderr, flush=True)
        srv.close()
        del pool, srv
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        tx.tx_pool_trim()
    ok = [r["speed"] for r in runs if r["p99_below_block"] and r["source"] == "host"]
    dev = [r["value"] for r in runs if r["source"] == "device"]
    host = [r["value"] for r in runs if r["source"] == "host"]
    return {"workload": "served-4096", "beams": nbeams, "lanes": lanes, "slots": slots,
            "block_duration_ms": t_blk * 1e3, "unit": "DM-trial samples/s", "runs": runs,
            "max_host_speed_p99_below_block": max(ok) if ok else None,
            "value": max(dev) if dev else None, "value_host_pcie_inclusive": max(host) if host else None}


def octave_served_leg(torch, tx, synth, serve, runs_spec, lanes, max_slots, nbeams=32):
    """The multi-octave workload served and batched: 32 beams of 8192-channel
    blocks over 544-1088 MHz (65536 samples, 10.03 s each, 8192 trials to
    DM 5000, widths to 1024) at Poisson arrivals, each beam's 343278-sample
    overlap history resident on the device (3.35 GB per beam), admission
    bounded by the device memory left; blocks already in device memory.  The
    first 5.2 blocks of a beam only fill its history."""
    wl = synth.workload("octave-8192")
    plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    nchan, nt = plan.nchan, wl.nt
    t_blk = nt * wl.tsamp
    pool = [synth.device_normal_u8(torch, nchan, nt, 5000 + i) for i in range(4)]
    srv = serve.Server([plan] * nbeams, nt, wl.widths, gamma=wl.gamma, cap=4096, lanes=lanes, max_slots=max_slots,
                       graph=True, source="device", keep=())
    runs = []
    for speed, nblocks in runs_spec:
        for st in srv.streams:
            st.reset()
        arr = synth.poisson_arrivals(nbeams, nblocks, t_blk, speed, 50 + speed)
        _, stats = srv.run(arr, lambda b, k: pool[(b * 5 + k) % len(pool)])
        emitted = stats.dm_samples
        apd = plan_adds(plan, nt) / (plan.ndm * nt)
        runs.append({"speed": speed, "blocks": stats.blocks, "batches": stats.batches,
                     "adds_per_s": stats.throughput * apd, "frac_of_add_peak": stats.throughput * apd / PEAK_ADD16,
                     "mean_batch": round(stats.mean_batch, 2), "p50_ms": stats.p50_s * 1e3,
                     "p99_ms": stats.p99_s * 1e3, "max_ms": stats.max_s * 1e3, "value": stats.throughput,
                     "dm_samples": emitted, "gpu_busy": stats.gpu_s / stats.wall_s if stats.wall_s > 0 else None,
                     "lane_overlap": stats.lane_s / stats.gpu_s if stats.gpu_s > 0 else None,
                     "p99_below_block": stats.p99_s < t_blk})
        print(f"octave served: {json.dumps(runs[-1])}", file=sys.stderr, flush=True)
    slots = srv.slots
    srv.close()
    del pool, srv
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    tx.tx_pool_trim()
    return {"workload": "octave-8192 served", "beams": nbeams, "lanes": lanes, "slots": slots,
            "block_duration_ms": t_blk * 1e3, "unit": "DM-trial samples/s", "source": "device", "runs": runs,
            "value": max(r["value"] for r in runs) if runs else None,
            "p99_below_block_all": all(r["p99_below_block"] for r in runs)}


def latency_leg(torch, tx, synth, reps=200):
    """The single-beam configuration at its small size (plain-256: 256
    channels, 128 trials, 8192 samples of 306.24 us): one block's latency
    from launch to peaks and candidate count in host memory, through
    tx_dedisperse and tx_candidates on a resident block (launch-bound at this
    size)."""
    wl = synth.workload("plain-256")
    plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    nt = wl.nt
    pitch = (nt + plan.overlap + 255) // 256 * 256
    d_in = synth.device_normal_u8(torch, plan.nchan, pitch, wl.seed, pulses=place_pulses(plan, wl, synth))
    y = torch.empty((plan.ndm, nt), dtype=torch.int32, device="cuda")
    cands = torch.empty((1 << 14, 3), dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    peaks = (torch.empty(plan.ndm, dtype=torch.float64, device="cuda"),
             torch.empty(plan.ndm, dtype=torch.int32, device="cuda"),
             torch.empty(plan.ndm, dtype=torch.int64, device="cuda"))
    host_snr = torch.empty(plan.ndm, dtype=torch.float64, pin_memory=True)
    host_cnt = torch.empty(1, dtype=torch.int64, pin_memory=True)
    stream = torch.cuda.current_stream()
    lat = []
    for k in range(reps + 10):
        t = time.perf_counter()
        tx.tx_dedisperse(plan, d_in, nt, y, stream=stream)
        tx.tx_candidates(y, nt, wl.widths, wl.gamma, cands, count, peaks=peaks, stream=stream)
        host_snr.copy_(peaks[0], non_blocking=True)
        host_cnt.copy_(count, non_blocking=True)
        stream.synchronize()
        if k >= 10:
            lat.append(time.perf_counter() - t)
    lat = np.array(lat) * 1e3
    best = int(np.argmax(host_snr.numpy()))
    return {"workload": "plain-256", "reps": reps, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "min_ms": float(lat.min()),
            "block_duration_ms": nt * wl.tsamp * 1e3, "dm_trial_samples_per_s": plan.ndm * nt / (np.median(lat) * 1e-3),
            "peak_dm_index": best, "peak_snr": float(host_snr[best]), "candidates": int(host_cnt.item())}


def cpu_baseline_extra(seconds):
    """The C oracle (as it is) at 1 thread and at every host thread, on
    bounded samples of the single-beam, paper-scale, served and multi-octave
    blocks (the first coarse groups of each DM grid, all of plain-256's;
    seeded uniform bytes, since the time of integer sums does not depend on
    the values): DM-trial samples/s of dedispersion + peaks + candidates.
    Context for the paper's one-core figure."""
    import oracle
    import synth
    from oracle import c_oracle as co
    nproc = co.max_threads()
    out = []
    for name, groups in (("plain-256", None), ("paper-4096", 1), ("served-4096", 2), ("octave-8192", 1)):
        wl = synth.workload(name)
        ref_g = oracle.group_size_rule(wl.freqs, wl.nsub, len(wl.dms))
        ntr = len(wl.dms) if groups is None else groups * ref_g
        dms = wl.dms[:ntr]
        ref = oracle.make_plan(wl.freqs, wl.tsamp, dms, wl.nsub, g=ref_g)
        nt = wl.nt
        x = synth.uniform_u8(len(wl.freqs), nt + ref.overlap, wl.seed)
        for threads in (1, nproc):
            t = time.perf_counter()
            reps = 0
            while True:
                y = co.dedisperse_subband(x, wl.freqs, wl.tsamp, dms, wl.nsub, ref_g, nt, threads=threads)
                co.boxcar_peaks(y, wl.widths, threads=threads)
                co.boxcar_candidates(y, wl.widths, wl.gamma, threads=threads)
                reps += 1
                dt = time.perf_counter() - t
                if dt > seconds / 8 or reps >= 50:
                    break
            out.append({"workload": name, "threads": threads, "trials": ntr, "of_trials": len(wl.dms),
                        "samples": nt, "reps": reps, "seconds": round(dt, 2),
                        "value": reps * ntr * nt / dt, "unit": "DM-trial samples/s"})
            print(f"cpu: {json.dumps(out[-1])}", file=sys.stderr, flush=True)
        del x
    return {"kind": "oracle", "runs": out, "host_threads": nproc}


def norm_leg(torch, tx, synth, steps=10):
    """The normalised variant on the paper-scale block (Sec. 2.1 then the
    path in float32): exact per-channel power sums on the device, inverse-
    variance weights on the host, float32 two-stage dedispersion and the
    float64 matched filter with candidates.  Timed per step (weights, upload,
    dedispersion, candidates); per-kernel times from events."""
    wl = synth.workload("paper-4096")
    plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    nchan, nt, ndm = plan.nchan, wl.nt, plan.ndm
    n = nt + plan.overlap
    pitch = (n + 255) // 256 * 256
    d_in = synth.device_normal_u8(torch, nchan, pitch, wl.seed, pulses=place_pulses(plan, wl, synth))
    sums = torch.empty((nchan, 4), dtype=torch.int64, device="cuda")
    y = torch.empty((ndm, nt), dtype=torch.float32, device="cuda")
    cap = 1 << 20
    cands = torch.empty((cap, 3), dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    peaks = (torch.empty(ndm, dtype=torch.float64, device="cuda"),
             torch.empty(ndm, dtype=torch.int32, device="cuda"),
             torch.empty(ndm, dtype=torch.int64, device="cuda"))
    d_s = torch.empty(nchan, dtype=torch.float32, device="cuda")
    d_o = torch.empty(nchan, dtype=torch.float32, device="cuda")

    def step():
        tx.tx_channel_power_sums(d_in, nchan, n, sums)
        scale, offset = tx.tx_norm_weights(sums.cpu().numpy(), n, tx.TX_WEIGHT_INVERSE_VAR)
        d_s.copy_(torch.from_numpy(scale))
        d_o.copy_(torch.from_numpy(offset))
        tx.tx_dedisperse_norm(plan, d_in, nt, d_s, d_o, y)
        tx.tx_candidates_f32(y, nt, wl.widths, wl.gamma, cands, count, peaks=peaks)

    step()
    torch.cuda.synchronize()
    for k in (tx.TX_KERNEL_STAGE1, tx.TX_KERNEL_STAGE2, tx.TX_KERNEL_BOXCAR):
        tx.tx_profile_collect(k)
    tx.tx_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    tx.tx_profile_enable(False)
    kern = {}
    for name, k in (("stage1", tx.TX_KERNEL_STAGE1), ("stage2", tx.TX_KERNEL_STAGE2), ("boxcar", tx.TX_KERNEL_BOXCAR)):
        ms, nl = tx.tx_profile_collect(k)
        kern[name] = {"avg_ms": ms / max(nl, 1), "launches": nl}
    best = int(torch.argmax(peaks[0]).item())
    # float operations: a fused multiply-add and an add per first-stage term,
    # an add per second-stage term
    flops = 3 * plan.ngroups * nchan * nt + ndm * plan.nsub * nt
    t12 = (kern["stage1"]["avg_ms"] + kern["stage2"]["avg_ms"]) * 1e-3
    out = {"workload": "paper-4096 normalised (inverse-variance weights), float32", "ms_per_block": dt * 1e3,
           "dm_trial_samples_per_s": ndm * nt / dt, "kernels_ms": kern, "candidates": int(count.item()),
           "peak_dm_index": best, "peak_snr": float(peaks[0][best].item()),
           "roofline": {"bound": "alu", "achieved": round(flops / t12 / 1e12, 3), "peak": 157.3,
                        "unit": "TFLOP/s (fp32 vector)", "frac": round(flops / t12 / 157.3e12, 4),
                        "flops_per_block": flops}}
    del d_in, y, cands
    torch.cuda.empty_cache()
    tx.tx_pool_trim()
    return out


def serve_mod():
    from paper_2401_13834_amd import serve
    return serve


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper-4096")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-beam batched launch")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--batched-no-tune", action="store_true",
                    help="run the batched leg with each plan's own sub-band count and tiles only")
    ap.add_argument("--no-served", action="store_true", help="skip the served-stream runs")
    ap.add_argument("--served-runs", default="host:1:2,host:8:9,host:24:13,device:24:13,device:48:25",
                    help="source:speed:blocks-per-beam of the served runs (source host or device)")
    ap.add_argument("--served-lanes", type=int, default=2)
    ap.add_argument("--served-slots", type=int, default=32)
    ap.add_argument("--no-transpose", action="store_true", help="skip the time-major ingest leg")
    ap.add_argument("--no-ranges", action="store_true", help="skip the multi-range (downsampled) plan leg")
    ap.add_argument("--no-cluster", action="store_true", help="skip the DM-time clustering leg")
    ap.add_argument("--no-stats", action="store_true", help="skip the channel statistics leg")
    ap.add_argument("--no-octave", action="store_true", help="skip the served multi-octave leg")
    ap.add_argument("--octave-runs", default="8:9,24:9",
                    help="speed:blocks-per-beam of the served multi-octave runs")
    ap.add_argument("--no-latency", action="store_true", help="skip the plain-256 latency leg")
    ap.add_argument("--no-norm", action="store_true", help="skip the normalised (float32) variant leg")
    ap.add_argument("--no-cpu-extra", action="store_true",
                    help="skip the CPU oracle at 1 thread and on the other workloads")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed steps, copy the DM x time array once (a plain copy of known size "
                         "whose HBM counters scale the kernels' counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs the hot path on a single MI355X "
              "(beams shard across GPUs with no exchange, so the one-GPU rate is the per-GPU rate).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2401_13834_amd as tx

    wl = synth.workload(args.workload)
    plan = tx.tx_plan(wl.freqs, wl.tsamp, wl.dms, wl.nsub)
    nchan, ndm, nt = len(wl.freqs), plan.ndm, wl.nt
    pitch = (nt + plan.overlap + 255) // 256 * 256
    d_in = make_input(torch, plan, wl, synth, pitch)
    # host copy of the block for the CPU baseline (the same bytes)
    x = None if args.no_cpu_baseline else d_in[:, :nt + plan.overlap].cpu().numpy()
    y = torch.empty((ndm, nt), dtype=torch.int32, device="cuda")
    cap = 1 << 20
    cands = torch.empty((cap, 3), dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    peaks = (torch.empty(ndm, dtype=torch.float64, device="cuda"),
             torch.empty(ndm, dtype=torch.int32, device="cuda"),
             torch.empty(ndm, dtype=torch.int64, device="cuda"))
    stream = torch.cuda.current_stream()

    def step():
        tx.tx_dedisperse(plan, d_in, nt, y, stream=stream)
        tx.tx_candidates(y, nt, wl.widths, wl.gamma, cands, count, peaks=peaks, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for k in (tx.TX_KERNEL_STAGE1, tx.TX_KERNEL_STAGE2, tx.TX_KERNEL_BOXCAR):
        tx.tx_profile_collect(k)
    tx.tx_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tx.tx_profile_enable(False)
    kern = {}
    for name, k in (("stage1", tx.TX_KERNEL_STAGE1), ("stage2", tx.TX_KERNEL_STAGE2),
                    ("boxcar", tx.TX_KERNEL_BOXCAR)):
        ms, n = tx.tx_profile_collect(k)
        kern[name] = {"avg_ms": ms / max(n, 1), "launches": n}
    ncand = int(count.item())
    if args.copy_probe:
        y2 = torch.empty_like(y)
        y2.copy_(y)
        torch.cuda.synchronize()
        del y2

    value = ndm * nt * args.steps / elapsed
    adds1 = plan.ngroups * nchan * nt                 # first stage: N_c * N_f * T additions
    adds2 = ndm * plan.nsub * nt                      # second stage: N_DM * nsub * T additions
    t1 = kern["stage1"]["avg_ms"] * 1e-3
    achieved = adds1 / t1 / 1e12
    traffic = load_traffic("stage1", args.workload)
    # The first stage's inner loop, per 4 byte-adds of one channel: 3 VALU ops
    # (byte align, byte permute, half of each of two 3-input adds) and
    # (Q + 1) / Q 4-byte LDS reads issued as paired reads (Q = output dwords
    # per lane of the tile variant in use).  Its two ceilings: 256 CUs x 4
    # SIMDs x 16 lanes x 2.4 GHz lane-ops at 4/3 adds each, and paired LDS
    # reads at the rate measured on this part.
    q1 = tx.tx_tile_variants(1)[plan.resolved_tiles(nt)[0]][0] // 256
    valu_ceiling = 256 * 4 * 16 * 2.4e9 * 4 / 3 / 1e12
    valu_ceiling_measured = 256 * MEASURED_VOP3_PER_CLK_CU * 2.4e9 * 4 / 3 / 1e12
    lds_ceiling = MEASURED_PAIRED_LDS_B_PER_CLK_CU * 256 * 2.4e9 / ((q1 + 1) / q1) / 1e12
    loop_ceiling = min(valu_ceiling, lds_ceiling)
    roofline = {"bound": "alu", "kernel": "stage1", "achieved": round(achieved, 3),
                "peak": round(PEAK_ADD16 / 1e12, 3), "unit": "Tadd/s", "frac": round(achieved * 1e12 / PEAK_ADD16, 4),
                "traffic": traffic,
                # HBM rate of the same launches (counter bytes / event time), against 8 TB/s
                "hbm_GBps": None if traffic is None else round(traffic / t1 / 1e9, 1),
                "hbm_frac": None if traffic is None else round(traffic / t1 / 8e12, 4),
                "loop_ceiling_Tadd_s": round(loop_ceiling, 2),
                "loop_bound": "valu" if valu_ceiling <= lds_ceiling else "lds",
                "loop_ceiling_frac": round(achieved / loop_ceiling, 4),
                "loop_ceiling_measured_Tadd_s": round(min(valu_ceiling_measured, lds_ceiling), 2),
                "loop_ceiling_measured_frac": round(achieved / min(valu_ceiling_measured, lds_ceiling), 4)}

    # The other two kernels of the step against HBM: counter bytes per launch
    # (committed rocprofv3 summary, current source only) over event time.
    def hbm_entry(k, adds=None):
        t = kern[k]["avg_ms"] * 1e-3
        tr = load_traffic(k, args.workload)
        e = {"ms": round(t * 1e3, 4), "traffic": tr,
             "hbm_GBps": None if tr is None else round(tr / t / 1e9, 1),
             "hbm_frac": None if tr is None else round(tr / t / 8e12, 4),
             "copy_frac": None if tr is None else round(tr / t / MEASURED_COPY_BYTES_PER_S, 4)}
        rw = load_traffic(k, args.workload, split=True)
        if rw is not None:
            # Time to stream the kernel's own counter bytes at the measured
            # read and write rates, and the fraction of the launch time it is.
            floor = rw[0] / MEASURED_READ_BYTES_PER_S + rw[1] / MEASURED_WRITE_BYTES_PER_S
            e.update({"stream_floor_ms": round(floor * 1e3, 4), "stream_frac": round(floor / t, 4)})
        if adds is not None:
            e.update({"achieved_Tadd_s": round(adds / t / 1e12, 3), "add_frac": round(adds / t / PEAK_ADD16, 4)})
        return e

    out = {
        "metric": "dedispersed DM-trial samples/s (plain one-beam-per-launch path)",
        "value": value,
        "unit": "DM-trial samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": value / PAPER_DM_SAMPLES_PER_S if args.workload == "paper-4096" else None,
        "vs_baseline_ref": "paper, Sec. 3: 4096 channels x 4096 trials at 153 us dedispersed in real time on one "
                           "i7-10750H core, i.e. >= 2.68e7 DM-trial samples/s (a bound on other hardware)",
        "dtype": "int32",
        "input_dtype": "u8",
        "data": "synthetic",
        "config": {"workload": args.workload, "nchan": nchan, "ndm": ndm, "nt": nt, "nsub": plan.nsub,
                   "dms_per_group": plan.g, "tsamp_us": wl.tsamp * 1e6, "widths": f"1..{wl.widths[-1]}",
                   "gamma": wl.gamma, "parallelism": "single-gpu"},
        "block_latency_ms": elapsed / args.steps * 1e3,
        "block_duration_ms": nt * wl.tsamp * 1e3,
        "kernels_ms": kern,
        "adds_per_step": adds1 + adds2,
        "candidates_last_step": ncand,
        "roofline": roofline,
        "roofline_kernels": {"stage2": hbm_entry("stage2", adds2), "boxcar": hbm_entry("boxcar")},
    }
    del d_in, y, cands
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    tx.tx_pool_trim()
    if not args.no_transpose:
        out["transpose"] = transpose_leg(torch, tx, nchan, nt, plan.overlap)
        print(f"transpose: {json.dumps(out['transpose'])}", file=sys.stderr, flush=True)
    if not args.no_stats:
        out["channel_stats"] = stats_leg(torch, tx, nchan, nt + plan.overlap)
        print(f"channel_stats: {json.dumps(out['channel_stats'])}", file=sys.stderr, flush=True)
    if not args.no_ranges:
        out["ranges"] = ranges_leg(torch, tx, synth)
        print(f"ranges: {json.dumps(out['ranges'])}", file=sys.stderr, flush=True)
    if not args.no_cluster:
        out["cluster"] = cluster_leg(torch, tx, synth)
        print(f"cluster: {json.dumps(out['cluster'])}", file=sys.stderr, flush=True)
    if not args.no_batched:
        out["batched"] = batched_leg(torch, tx, synth, args.batched_steps, tune=not args.batched_no_tune)
        print(f"batched: {json.dumps(out['batched'])}", file=sys.stderr, flush=True)
    if not args.no_served:
        serve = serve_mod()
        spec = []
        for item in args.served_runs.split(","):
            if item:
                src, sp, nb = item.split(":")
                spec.append((src, int(sp), int(nb)))
        out["served"] = served_leg(torch, tx, synth, serve, spec, args.served_lanes, args.served_slots)
    if not args.no_octave:
        spec = []
        for item in args.octave_runs.split(","):
            if item:
                sp, nb = item.split(":")
                spec.append((int(sp), int(nb)))
        out["octave_served"] = octave_served_leg(torch, tx, synth, serve_mod(), spec, args.served_lanes,
                                                 args.served_slots)
    if not args.no_norm:
        out["normalised"] = norm_leg(torch, tx, synth)
        print(f"normalised: {json.dumps(out['normalised'])}", file=sys.stderr, flush=True)
    if not args.no_latency:
        out["latency_plain256"] = latency_leg(torch, tx, synth)
        print(f"latency: {json.dumps(out['latency_plain256'])}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, x, plan.g, args.cpu_seconds)
        if not args.no_cpu_extra:
            out["cpu_baseline"]["extra"] = cpu_baseline_extra(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
