"""Seeded synthetic inputs shared by the tests and the benchmark.

This module holds no dedispersion or matched-filter arithmetic.  It makes
filterbank blocks of quantised Gaussian noise, adds pulses at per-channel
sample positions that the caller computes, describes the benchmark workloads
(band, sampling time, DM grid, boxcar widths) and draws arrival times.
Everything is a pure function of its seed.

Noise recipe: ``x = clip(rint(mean + std * z + pulse), 0, 255)`` as uint8 with
``z`` standard normal float32 from ``numpy.random.Generator(PCG64(seed))``,
drawn row block by row block (64 channels at a time).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ROWS_PER_DRAW = 64


def _apply_pulses(z, row0, pulses):
    """Add pulse amplitudes to the float rows ``z`` (channels row0 .. row0+len)."""
    rows, nsamp = z.shape
    for start, width, amp in pulses:
        start = np.asarray(start, dtype=np.int64)
        amp_arr = np.broadcast_to(np.asarray(amp, dtype=np.float64), start.shape)
        for r in range(rows):
            ch = row0 + r
            a = int(start[ch])
            b = min(a + int(width), nsamp)
            a = max(a, 0)
            if a < b:
                z[r, a:b] += np.float32(amp_arr[ch])


def normal_u8(nchan, nsamp, seed, *, mean=128.0, std=16.0, pulses=()):
    """[nchan, nsamp] uint8 block of clipped, rounded N(mean, std^2) noise.

    ``pulses`` is a sequence of (start[nchan], width, amplitude) where
    ``start[ch]`` is the first sample of the pulse in channel ``ch`` and the
    amplitude (scalar or per channel) is added before rounding."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((nchan, nsamp), dtype=np.uint8)
    for r0 in range(0, nchan, ROWS_PER_DRAW):
        r1 = min(nchan, r0 + ROWS_PER_DRAW)
        z = rng.standard_normal((r1 - r0, nsamp), dtype=np.float32)
        z *= np.float32(std)
        z += np.float32(mean)
        _apply_pulses(z, r0, pulses)
        np.rint(z, out=z)
        np.clip(z, 0, 255, out=z)
        out[r0:r1] = z.astype(np.uint8)
    return out


def pooled_normal_u8(nchan, nsamp, seed, *, pool=64, mean=128.0, std=16.0, pulses=()):
    """Like ``normal_u8`` but fast for large blocks: ``pool`` noise rows are
    drawn once and channel ``ch`` is pool row ``k[ch]`` rotated by ``s[ch]``
    samples (``k`` and ``s`` drawn from the same seed).  Channels are then not
    independent, which matters for statistics but not for throughput or
    exactness checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pool = min(pool, nchan)
    base = rng.standard_normal((pool, nsamp), dtype=np.float32)
    base *= np.float32(std)
    base += np.float32(mean)
    k = rng.integers(0, pool, size=nchan)
    s = rng.integers(0, nsamp, size=nchan)
    out = np.empty((nchan, nsamp), dtype=np.uint8)
    for r0 in range(0, nchan, ROWS_PER_DRAW):
        r1 = min(nchan, r0 + ROWS_PER_DRAW)
        z = np.stack([np.roll(base[k[c]], int(s[c])) for c in range(r0, r1)])
        _apply_pulses(z, r0, pulses)
        np.rint(z, out=z)
        np.clip(z, 0, 255, out=z)
        out[r0:r1] = z.astype(np.uint8)
    return out


def uniform_u8(nchan, nsamp, seed):
    """[nchan, nsamp] uint8, every value 0..255 equally likely."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 256, size=(nchan, nsamp), dtype=np.uint8)


def uniform_i32(nrows, nsamp, seed, lo, hi):
    """[nrows, nsamp] int32 uniform on [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=(nrows, nsamp), dtype=np.int64).astype(np.int32)


def band_centres(f_top, f_bottom, nchan):
    """Centre frequencies (MHz) of ``nchan`` equal channels filling the band,
    highest first (the usual filterbank order with a negative channel step)."""
    bw = (float(f_top) - float(f_bottom)) / nchan
    return np.array([float(f_top) - (c + 0.5) * bw for c in range(nchan)], dtype=np.float64)


def pow2_widths(wmax):
    """1, 2, 4, ..., wmax."""
    out, w = [], 1
    while w <= wmax:
        out.append(w)
        w *= 2
    return out


@dataclass
class Workload:
    name: str
    freqs: np.ndarray
    tsamp: float
    dms: np.ndarray
    nsub: int
    nt: int
    widths: list
    seed: int
    gamma: float = 6.0
    pulses: list = field(default_factory=list)   # (dm, t, width, snr-or-amp spec)


def workload(name):
    """The benchmark workloads, by name.

    * ``plain-256``: 256 channels over 856-1712 MHz, 306.24 us, 8192 output
      samples, 128 DM trials 0..508 step 4, 16 sub-bands, widths 1..64, one
      pulse (DM 200, width 4, +6 sigma per channel = +96 counts, t = 4000).
    * ``paper-4096``: 4096 channels over 856-1712 MHz, 153.12 us, 65536 output
      samples, 4096 DM trials 0..2047.5 step 0.5, 64 sub-bands, widths 1..512,
      ten pulses (random DM, width 1..32, integrated S/N 3..10).
    * ``served-4096``: the served-stream block: 4096 channels, 153.12 us, 32768
      samples, 2048 DM trials 0..1023.5, 64 sub-bands, widths 1..512.
    * ``octave-8192``: 8192 channels over 544-1088 MHz, 153.12 us, 65536
      samples, 8192 trials evenly over 0..5000, 64 sub-bands, widths 1..1024.
    """
    if name == "plain-256":
        return Workload(name, band_centres(1712.0, 856.0, 256), 306.24e-6,
                        np.arange(128, dtype=np.float64) * 4.0, 16, 8192, pow2_widths(64), 1,
                        pulses=[("amp", 200.0, 4000, 4, 96.0)])
    if name == "paper-4096":
        rng = np.random.Generator(np.random.PCG64(2002))
        pulses = []
        slots = rng.permutation(10)
        for k in range(10):
            dm = float(rng.uniform(0.0, 2047.5))
            w = int(rng.integers(1, 33))
            snr = float(rng.uniform(3.0, 10.0))
            t = int(slots[k]) * 6400 + 1000          # non-overlapping start times
            pulses.append(("snr", dm, t, w, snr))
        return Workload(name, band_centres(1712.0, 856.0, 4096), 153.12e-6,
                        np.arange(4096, dtype=np.float64) * 0.5, 64, 65536, pow2_widths(512), 2,
                        pulses=pulses)
    if name == "served-4096":
        return Workload(name, band_centres(1712.0, 856.0, 4096), 153.12e-6,
                        np.arange(2048, dtype=np.float64) * 0.5, 64, 32768, pow2_widths(512), 4)
    if name == "octave-8192":
        return Workload(name, band_centres(1088.0, 544.0, 8192), 153.12e-6,
                        np.linspace(0.0, 5000.0, 8192), 64, 65536, pow2_widths(1024), 5,
                        pulses=[("snr-index", 2500.0, 30000, 8, 12.0)])
    raise KeyError(name)


def dm_ranges(name):
    """DM ranges of a multi-range plan over a named workload's block, as
    (dms, downsampling factor) pairs.

    * ``ranges-4096``: the ``paper-4096`` block (4096 channels over
      856-1712 MHz, 153.12 us, 65536 samples, 64 sub-bands) searched over
      DM 0..2046 in three ranges, coarser in DM and time as DM grows:
      0..511.5 step 0.5 at full rate, 512..1023 step 1 downsampled by 2,
      1024..2046 step 2 downsampled by 4 (2048 trials).
    """
    if name == "ranges-4096":
        return [(np.arange(1024, dtype=np.float64) * 0.5, 1),
                (512.0 + np.arange(512, dtype=np.float64), 2),
                (1024.0 + 2.0 * np.arange(512, dtype=np.float64), 4)]
    raise KeyError(name)


def pulse_amplitude(spec, width, nchan, std=16.0):
    """Per-channel amplitude for a pulse spec: ``("amp", ..., a)`` is a fixed
    amplitude; ``("snr", ..., s)`` spreads an integrated S/N ``s`` evenly over
    channels and samples, a = std * s / sqrt(nchan * width)."""
    kind = spec[0]
    if kind == "amp":
        return float(spec[-1])
    return float(std * spec[-1] / np.sqrt(nchan * width))


def spectral_amplitudes(freqs, f0, index, scale):
    """Per-channel amplitude ``scale * (f / f0) ** index`` (a power-law spectrum)."""
    return scale * (np.asarray(freqs, dtype=np.float64) / f0) ** index


# The octave workload's pulse spectrum: flux proportional to f ** -1.5 around 816 MHz.
SPECTRAL_F0_MHZ = 816.0
SPECTRAL_INDEX = -1.5


def index_pulse_amplitudes(freqs, width, snr, std=16.0, f0=SPECTRAL_F0_MHZ, index=SPECTRAL_INDEX):
    """Per-channel amplitudes of a power-law pulse whose equal-weight
    integrated S/N is ``snr``: amplitudes a_c proportional to (f_c/f0)**index,
    scaled so that sum_c a_c = std * snr * sqrt(nchan) / sqrt(width).  (A
    window of ``width`` samples then holds width * sum_c a_c of signal over a
    noise of std * sqrt(nchan * width); with a flat spectrum this is
    ``pulse_amplitude``'s a = std * snr / sqrt(nchan * width) per channel.)"""
    freqs = np.asarray(freqs, dtype=np.float64)
    shape = spectral_amplitudes(freqs, f0, index, 1.0)
    return shape * (std * snr * np.sqrt(freqs.size) / np.sqrt(width) / shape.sum())


def place_pulses(wl, delays):
    """(start[nchan], width, amplitude) of every pulse of workload ``wl``, as
    ``normal_u8`` and ``device_normal_u8`` take them.  ``delays(dm)`` returns
    the per-channel delay in samples of a DM (from the caller's plan, so that
    the injection uses the plan's own rounding); a pulse at time t starts at
    t + delays(dm)[c] in channel c.  Specs: ``("amp", dm, t, w, a)`` a fixed
    amplitude, ``("snr", dm, t, w, s)`` a flat spectrum of integrated S/N s,
    ``("snr-index", dm, t, w, s)`` the power-law spectrum of
    ``index_pulse_amplitudes`` with integrated S/N s."""
    nchan = len(wl.freqs)
    out = []
    for spec in wl.pulses:
        kind, dm, t0, w = spec[0], spec[1], spec[2], spec[3]
        start = int(t0) + np.asarray(delays(dm), dtype=np.int64)
        if kind == "snr-index":
            amp = index_pulse_amplitudes(wl.freqs, w, spec[4])
        else:
            amp = pulse_amplitude(spec, w, nchan)
        out.append((start, w, amp))
    return out


def device_normal_u8(torch, nchan, nsamp, seed, *, device="cuda", mean=128.0, std=16.0, pulses=(), rows=256):
    """Same recipe as ``normal_u8`` drawn on the device with torch's generator
    (a different sequence of numbers than ``normal_u8`` for the same seed),
    for blocks too large to draw on the host.  ``pulses`` as in ``normal_u8``;
    ``torch.round`` rounds half to even like ``np.rint``."""
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    out = torch.empty((nchan, nsamp), dtype=torch.uint8, device=device)
    for r0 in range(0, nchan, rows):
        r1 = min(nchan, r0 + rows)
        z = torch.randn((r1 - r0, nsamp), generator=gen, device=device, dtype=torch.float32)
        z.mul_(float(std)).add_(float(mean))
        for start, width, amp in pulses:
            st = np.asarray(start, dtype=np.int64)[r0:r1]
            a = np.broadcast_to(np.asarray(amp, dtype=np.float64), (nchan,))[r0:r1]
            cols = st[:, None] + np.arange(int(width), dtype=np.int64)[None, :]
            rr = np.broadcast_to(np.arange(r1 - r0, dtype=np.int64)[:, None], cols.shape)
            ok = (cols >= 0) & (cols < nsamp)
            vals = np.broadcast_to(a.astype(np.float32)[:, None], cols.shape)[ok]
            z.index_put_((torch.from_numpy(rr[ok]).to(device), torch.from_numpy(cols[ok]).to(device)),
                         torch.from_numpy(np.ascontiguousarray(vals)).to(device), accumulate=True)
        out[r0:r1] = z.round_().clamp_(0, 255).to(torch.uint8)
    return out


BATCHED_NCHAN = (1024, 2048, 4096)
BATCHED_NT = (16384, 32768, 49152, 65536)
BATCHED_NDM = (512, 1024, 1536, 2048, 3072, 4096)
BATCHED_DMMAX = (1000.0, 2000.0, 3000.0)


def batched_beams(n=64, seed=3):
    """The uneven batch: ``n`` beams over 856-1712 MHz at 153.12 us, each with
    a channel count, block length, DM grid (``ndm`` trials evenly over
    0..dm_max) and 0-5 pulses (DM uniform on the grid's range, width 1..32,
    integrated S/N 3..10, start uniform in the block) drawn from ``seed``.
    ``nsub`` is 0: the plan picks it."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(n):
        nchan = int(rng.choice(BATCHED_NCHAN))
        nt = int(rng.choice(BATCHED_NT))
        ndm = int(rng.choice(BATCHED_NDM))
        dmmax = float(rng.choice(BATCHED_DMMAX))
        pulses = []
        for _ in range(int(rng.integers(0, 6))):
            w = int(rng.integers(1, 33))
            pulses.append(("snr", float(rng.uniform(0.0, dmmax)), int(rng.integers(0, nt - w)), w,
                           float(rng.uniform(3.0, 10.0))))
        out.append(Workload(f"batched-{b}", band_centres(1712.0, 856.0, nchan), 153.12e-6,
                            np.linspace(0.0, dmmax, ndm), 0, nt, pow2_widths(512), 1000 * seed + b, pulses=pulses))
    return out


def poisson_arrivals(nbeams, nblocks, period_s, speed, seed):
    """Arrival times [nbeams, nblocks] in seconds: each beam starts at a
    uniform time in [0, period) and then waits exponential gaps of mean
    period / speed between blocks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    start = rng.uniform(0.0, period_s, size=nbeams)
    gaps = rng.exponential(period_s / speed, size=(nbeams, nblocks))
    gaps[:, 0] = 0.0
    return start[:, None] + np.cumsum(gaps, axis=1)


def plane_points(n, ndm, nt, seed, blob_frac=0.7, blob_size=200, spread=3):
    """``n`` distinct DM-time points (d, t, width, snr) as a thresholded plane
    holds them: about ``blob_frac`` of them in blobs of about ``blob_size``
    points around random (d, t) (a pulse seen at neighbouring trials and
    times, +-spread trials and +-4 spread samples), the rest scattered
    uniformly; widths 1..64, S/N uniform in [6, 20).  Returned as an int64
    array [n, 3] in the record layout of the candidate list
    (d | width << 32, time, snr bits), rows in random order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = np.empty(0, dtype=np.int64)
    n_blob = int(n * blob_frac)
    while keys.size < n_blob:
        nb = max(1, (n_blob - keys.size) // blob_size + 1)
        d0 = rng.integers(0, ndm, size=nb)
        t0 = rng.integers(0, nt, size=nb)
        d = (np.repeat(d0, blob_size) + rng.integers(-spread, spread + 1, size=nb * blob_size))
        t = (np.repeat(t0, blob_size) + rng.integers(-4 * spread, 4 * spread + 1, size=nb * blob_size))
        ok = (d >= 0) & (d < ndm) & (t >= 0) & (t < nt)
        keys = np.unique(np.concatenate([keys, d[ok] * nt + t[ok]]))
    keys = rng.permutation(keys)[:n_blob] if keys.size > n_blob else keys
    while keys.size < n:
        extra = rng.integers(0, ndm, size=n - keys.size) * nt + rng.integers(0, nt, size=n - keys.size)
        keys = np.unique(np.concatenate([keys, extra]))
    keys = keys[rng.permutation(keys.size)[:n]]
    d, t = keys // nt, keys % nt
    w = rng.integers(1, 65, size=n).astype(np.int64)
    snr = rng.uniform(6.0, 20.0, size=n)
    out = np.empty((n, 3), dtype=np.int64)
    out[:, 0] = d | (w << 32)
    out[:, 1] = t
    out[:, 2] = snr.view(np.int64)
    return out
