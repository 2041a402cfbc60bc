"""Serving loop: continuous batching of streaming beam blocks over the C ABI.

Every beam keeps its plan and its overlap history (a ``tx.Stream``, the
buffer of the paper's "shift data" step, Sec. 2.3) resident on the device
between blocks.  Blocks arrive at host-clock times.  The loop:

* releases blocks whose arrival time has passed into a ready queue (arrival
  order; one beam's blocks stay in order);
* admits ready blocks into a free *lane* as soon as one exists, at most one
  block per beam per lane and at most ``slots`` blocks per lane, where
  ``slots`` follows from the device memory left after the resident rings
  (memory-bounded admission);
* copies host blocks to device staging slots on a copy stream, so uploads
  overlap the kernels of lanes already queued;
* runs each lane as one ``tx.Batch`` launch (persistent kernels over a device
  job table, replayed as a HIP graph) on the lane's own compute stream, then
  copies the lane's peaks and candidate lists back in one transfer;
* harvests lanes in completion order; a block's latency runs from its arrival
  to the moment its candidates are host-visible.

Every lane has its own compute stream, so the work of lanes admitted while
others run overlaps on the device.  One beam's blocks must still update its
overlap history in order: a lane whose beam's previous block is in another
lane still in flight waits for that lane's kernels (a per-beam event) before
its own start, and only then.
"""

import collections
import dataclasses
import time

import numpy as np

import paper_2401_13834_amd as tx


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the serving loop needs a HIP device")
    return torch


def _round_up(v, m):
    return (v + m - 1) // m * m


@dataclasses.dataclass
class BlockResult:
    beam: int
    index: int
    arrival: float          # seconds from the start of the run
    done: float             # candidates host-visible, seconds from the start
    n_out: int              # output samples per trial (0 while a stream primes)
    ndm: int
    count: int              # candidates found (may exceed the lane's capacity)
    snr: np.ndarray = None
    width: np.ndarray = None
    time: np.ndarray = None
    cands: np.ndarray = None
    dmt: np.ndarray = None

    @property
    def latency(self):
        return self.done - self.arrival


@dataclasses.dataclass
class ServeStats:
    blocks: int
    batches: int
    mean_batch: float
    dm_samples: int
    wall_s: float
    gpu_s: float            # time with at least one lane's work on the device
    lane_s: float           # summed time of the lanes' work (exceeds gpu_s when lanes overlap)
    p50_s: float
    p99_s: float
    max_s: float
    slots: int
    lanes: int

    @property
    def throughput(self):
        """Dedispersed DM-trial samples per second of wall time."""
        return self.dm_samples / self.wall_s if self.wall_s > 0 else 0.0


class _Lane:
    pass


class Server:
    """Continuous-batching server for ``len(plans)`` beams.

    plans:     one ``tx.Plan`` per beam (beams may share a plan object).
    block_nt:  samples per arriving block (every beam).
    widths, gamma, cap: boxcar widths, candidate threshold and the candidate
               capacity per block.
    lanes:     batches that may be queued on the device at once.
    max_slots: upper bound on blocks per lane; the device memory left after
               the rings (``mem_budget`` bytes, default: free memory less
               ``mem_reserve``) may lower it.
    source:    "host" (blocks arrive in host memory and are uploaded on a copy
               stream) or "device" (blocks are already in device memory).
    keep:      which per-block results to keep: any of "peaks", "cands",
               "dmt" (the last copies the DM x time array back: tests only;
               ``dmt_rows`` limits it to those trial rows).
    """

    def __init__(self, plans, block_nt, widths, *, gamma=6.0, cap=4096, lanes=2, max_slots=32, mem_budget=None,
                 mem_reserve=4 << 30, graph=True, source="host", keep=("peaks", "cands"), dmt_rows=None):
        torch = _torch()
        if source not in ("host", "device"):
            raise ValueError("source must be 'host' or 'device'")
        self.torch = torch
        self.plans = list(plans)
        self.nbeams = len(self.plans)
        self.block_nt = int(block_nt)
        self.widths = np.ascontiguousarray(widths, dtype=np.int32)
        self.gamma = float(gamma)
        self.cap = int(cap)
        self.source = source
        self.keep = set(keep)
        self.dmt_rows = None if dmt_rows is None else [int(r) for r in dmt_rows]
        self.graph = bool(graph)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        # resident state: one overlap ring per beam
        self.streams = [tx.Stream(p, self.block_nt) for p in self.plans]
        uniq = list({id(p): p for p in self.plans}.values())
        self.ndm_max = max(p.ndm for p in uniq)
        self.nchan_max = max(p.nchan for p in uniq)
        self.out_pitch = _round_up(max(self.block_nt, 2), 2)
        ws = max(p.ws_size(self.block_nt) for p in uniq)
        # per-slot result record: snr f64, time i64, width i32 (padded), count i64, candidates
        n = self.ndm_max
        self._o_snr = 0
        self._o_time = 8 * n
        self._o_width = 16 * n
        self._o_count = _round_up(20 * n, 8)
        self._o_cands = self._o_count + 8
        self.slot_bytes = _round_up(self._o_cands + 24 * self.cap, 256)
        per_slot = 4 * self.ndm_max * self.out_pitch + ws + self.slot_bytes
        if source == "host":
            per_slot += self.nchan_max * self.block_nt
        if mem_budget is None:
            free, _ = torch.cuda.mem_get_info(dev)
            mem_budget = max(0, free - mem_reserve)
        slots = min(int(max_slots), int(mem_budget // (lanes * per_slot)), self.nbeams)
        if slots < 1:
            raise MemoryError(f"device memory admits no block: {per_slot} bytes per slot, budget {mem_budget}")
        self.slots = slots
        self.per_slot_bytes = per_slot
        self.copy = torch.cuda.Stream(device=dev) if source == "host" else None
        self.lanes = []
        self.beam_event = {}     # beam -> event after the kernels of its latest launched block
        for _ in range(int(lanes)):
            ln = _Lane()
            ln.stream = torch.cuda.Stream(device=dev)
            ln.batch = tx.Batch(slots, graph=self.graph)
            for p in uniq:
                ln.batch.reserve(p, len(self.widths), self.block_nt, slots)
            ln.out = torch.empty((slots, self.ndm_max, self.out_pitch), dtype=torch.int32, device=dev)
            ln.res = torch.zeros(slots * self.slot_bytes, dtype=torch.uint8, device=dev)
            ln.host = torch.empty(slots * self.slot_bytes, dtype=torch.uint8, pin_memory=True)
            ln.stage = (torch.empty((slots, self.nchan_max, self.block_nt), dtype=torch.uint8, device=dev)
                        if source == "host" else None)
            ln.uploaded = torch.cuda.Event()
            ln.start = torch.cuda.Event(enable_timing=True)
            ln.done = torch.cuda.Event(enable_timing=True)
            ln.jobs = []
            self.lanes.append(ln)

    # -- one lane ----------------------------------------------------------
    def _views(self, ln, s, ndm):
        torch = self.torch
        base = s * self.slot_bytes
        r = ln.res
        snr = r[base + self._o_snr: base + self._o_snr + 8 * ndm].view(torch.float64)
        tim = r[base + self._o_time: base + self._o_time + 8 * ndm].view(torch.int64)
        wid = r[base + self._o_width: base + self._o_width + 4 * ndm].view(torch.int32)
        cnt = r[base + self._o_count: base + self._o_count + 8].view(torch.int64)
        cands = r[base + self._o_cands: base + self._o_cands + 24 * self.cap]
        return (snr, wid, tim), cands, cnt

    def _launch(self, ln, jobs, data_fn):
        torch = self.torch
        ln.jobs = jobs
        blocks = []
        st = ln.stream
        if self.source == "host":
            with torch.cuda.stream(self.copy):
                for s, (_, beam, k) in enumerate(jobs):
                    src = data_fn(beam, k)
                    nchan = self.plans[beam].nchan
                    dst = ln.stage[s, :nchan]
                    dst.copy_(src, non_blocking=True)
                    blocks.append(dst)
                ln.uploaded.record(self.copy)
            st.wait_event(ln.uploaded)
        else:
            blocks = [data_fn(beam, k) for (_, beam, k) in jobs]
        # One beam's blocks in order: wait for the kernels of each beam's
        # previous block where it ran on another lane's stream.
        waited = set()
        for (_, beam, _) in jobs:
            ev = self.beam_event.get(beam)
            if ev is not None and ev[0] is not ln and id(ev[1]) not in waited:
                st.wait_event(ev[1])
                waited.add(id(ev[1]))
        ln.batch.clear()
        for s, (_, beam, k) in enumerate(jobs):
            plan = self.plans[beam]
            peaks, cands, cnt = self._views(ln, s, plan.ndm)
            ln.batch.add_stream(self.streams[beam], blocks[s], self.block_nt, ln.out[s, :plan.ndm],
                                widths=self.widths, gamma=self.gamma, peaks=peaks, cands=cands, count=cnt)
        ln.start.record(st)
        ln.batch.launch(st)
        kern = torch.cuda.Event()
        kern.record(st)
        for (_, beam, _) in jobs:
            self.beam_event[beam] = (ln, kern)
        ln.n_out = [ln.batch.stream_output(s) for s in range(len(jobs))]
        used = len(jobs) * self.slot_bytes
        with torch.cuda.stream(st):
            ln.host[:used].copy_(ln.res[:used], non_blocking=True)
        ln.done.record(st)

    def _harvest(self, ln, now):
        out = []
        raw = ln.host.numpy()
        for s, (t_arr, beam, k) in enumerate(ln.jobs):
            plan = self.plans[beam]
            ndm = plan.ndm
            n_out = ln.n_out[s]
            base = s * self.slot_bytes
            r = BlockResult(beam, k, t_arr, now, n_out, ndm, 0)
            if n_out > 0:
                r.count = int(raw[base + self._o_count: base + self._o_count + 8].view(np.int64)[0])
                if "peaks" in self.keep:
                    r.snr = raw[base + self._o_snr: base + self._o_snr + 8 * ndm].view(np.float64).copy()
                    r.time = raw[base + self._o_time: base + self._o_time + 8 * ndm].view(np.int64).copy()
                    r.width = raw[base + self._o_width: base + self._o_width + 4 * ndm].view(np.int32).copy()
                if "cands" in self.keep:
                    r.cands = tx.parse_candidates(raw[base + self._o_cands: base + self._o_cands + 24 * self.cap],
                                                  r.count)
                if "dmt" in self.keep:
                    rows = slice(0, ndm) if self.dmt_rows is None else self.dmt_rows
                    r.dmt = ln.out[s, rows, :n_out].cpu().numpy()
            out.append(r)
        ln.gpu_s = ln.start.elapsed_time(ln.done) * 1e-3
        ln.span = (self._t_ref.elapsed_time(ln.start) * 1e-3, self._t_ref.elapsed_time(ln.done) * 1e-3)
        ln.jobs = []
        return out

    # -- the loop ----------------------------------------------------------
    def run(self, arrivals, data_fn, *, on_result=None, poll_s=5e-5):
        """Serve every block of ``arrivals`` and return (results, stats).

        arrivals: [nbeams, nblocks] arrival times in seconds from the start
                  (each row non-decreasing); block k of beam b is
                  ``data_fn(b, k)``: a uint8 tensor [nchan, block_nt], pinned
                  host memory for source "host", device memory otherwise.
        on_result: optional callable taking each BlockResult as it completes.
        """
        arrivals = np.asarray(arrivals, dtype=np.float64)
        if arrivals.ndim != 2 or arrivals.shape[0] != self.nbeams:
            raise ValueError("arrivals must be [nbeams, nblocks]")
        order = sorted((float(arrivals[b, k]), b, k) for b in range(self.nbeams) for k in range(arrivals.shape[1]))
        total = len(order)
        nxt = 0
        ready = collections.deque()
        inflight = collections.deque()
        free = list(self.lanes)
        results = []
        batches = 0
        gpu_s = 0.0
        torch = self.torch
        spans = []
        torch.cuda.synchronize()
        self._t_ref = torch.cuda.Event(enable_timing=True)
        self._t_ref.record(self.lanes[0].stream)
        self.beam_event = {}
        t0 = time.perf_counter()
        while len(results) < total:
            now = time.perf_counter() - t0
            while nxt < total and order[nxt][0] <= now:
                ready.append(order[nxt])
                nxt += 1
            for ln in [x for x in inflight if x.done.query()]:
                inflight.remove(ln)
                done_t = time.perf_counter() - t0
                got = self._harvest(ln, done_t)
                gpu_s += ln.gpu_s
                spans.append(ln.span)
                results.extend(got)
                if on_result is not None:
                    for r in got:
                        on_result(r)
                free.append(ln)
            if free and ready:
                jobs, seen, rest = [], set(), collections.deque()
                while ready and len(jobs) < self.slots:
                    item = ready.popleft()
                    if item[1] in seen:
                        rest.append(item)
                    else:
                        seen.add(item[1])
                        jobs.append(item)
                rest.extend(ready)
                ready = rest
                ln = free.pop()
                self._launch(ln, jobs, data_fn)
                inflight.append(ln)
                batches += 1
                continue
            if not inflight and not ready and nxt < total:
                time.sleep(min(max(order[nxt][0] - now, 0.0), 1e-3))
            else:
                time.sleep(poll_s)
        torch.cuda.synchronize()
        busy = 0.0                                  # time with at least one lane on the device
        end = -np.inf
        for a, b in sorted(spans):
            if a > end:
                busy += b - a
                end = b
            elif b > end:
                busy += b - end
                end = b
        lat = np.array([r.latency for r in results])
        first = order[0][0] if order else 0.0
        last = max((r.done for r in results), default=first)
        stats = ServeStats(blocks=total, batches=batches, mean_batch=total / max(batches, 1),
                           dm_samples=int(sum(r.ndm * r.n_out for r in results)), wall_s=last - first, gpu_s=busy,
                           lane_s=gpu_s,
                           p50_s=float(np.percentile(lat, 50)) if total else 0.0,
                           p99_s=float(np.percentile(lat, 99)) if total else 0.0,
                           max_s=float(lat.max()) if total else 0.0, slots=self.slots, lanes=len(self.lanes))
        results.sort(key=lambda r: (r.beam, r.index))
        return results, stats

    def close(self):
        for ln in self.lanes:
            ln.batch.close()
        for s in self.streams:
            s.close()
        self.lanes = []
        self.streams = []
