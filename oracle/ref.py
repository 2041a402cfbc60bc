"""Plain NumPy oracle: delay tables, brute-force and two-stage sub-band
dedispersion, boxcar S/N, peaks and threshold candidates.

Test infrastructure only (see the package docstring).  Every function restates
one step of the paper in the paper's order; nothing is blocked, fused or
reordered beyond what the definition states.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Dispersion constant e^2 / (2 pi m_e c) in s MHz^2 pc^-1 cm^3 (Sec. 2.3, Eq. 1).
# The paper prints the symbolic form only; this is the conventional value.
K_DM = 4.148808e3


# ---------------------------------------------------------------------------
# Delays and the plan (Sec. 2.3, Eq. 1 and the sub-band description)
# ---------------------------------------------------------------------------

def delay_samples(dm, f, fref, tsamp):
    """Integer delay, in samples, of frequency ``f`` (MHz) relative to ``fref``.

    Sec. 2.3, Eq. 1: tau = k DM (1/f^2 - 1/fref^2).  Reading: the delay in
    samples is rounded half-up, floor(tau / tsamp + 0.5), and the expression is
    evaluated in float64 in exactly this order:
    floor(((k * DM) * (1/(f*f) - 1/(fref*fref))) / tsamp + 0.5).
    ``dm`` and ``f`` broadcast against each other.
    """
    dm = np.asarray(dm, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    fref = np.float64(fref)
    inv_f2 = np.float64(1.0) / (f * f)
    inv_fref2 = np.float64(1.0) / (fref * fref)
    tau = (np.float64(K_DM) * dm) * (inv_f2 - inv_fref2)
    return np.floor(tau / np.float64(tsamp) + np.float64(0.5)).astype(np.int64)


def group_size_rule(freqs, nsub, ndm):
    """Number of fine DM trials per coarse group, g.

    The paper gives no rule (Sec. 2.3 only says the first stage uses a coarser
    DM grid, and Eq. 4 ties the smearing to the bandwidth).  Reading: the
    delay error that a coarse DM offset causes inside the widest sub-band must
    not exceed the full-band delay change of half a fine DM step, i.e.
    (g - 1) * a_max <= a_full / 2 with a = 1/f_lo^2 - 1/f_hi^2, so
    g = 1 + floor((a_full / a_max) / 2), capped at ``ndm``.  One channel per
    sub-band (or no frequency spread inside any sub-band) is exact for any g,
    and then g = ndm.
    """
    freqs = np.asarray(freqs, dtype=np.float64)
    nchan = freqs.shape[0]
    m = nchan // nsub
    fref = np.max(freqs)
    fmin = np.min(freqs)
    a_full = np.float64(1.0) / (fmin * fmin) - np.float64(1.0) / (fref * fref)
    a_max = np.float64(0.0)
    for s in range(nsub):
        sub = freqs[s * m:(s + 1) * m]
        hi = np.max(sub)
        lo = np.min(sub)
        a_s = np.float64(1.0) / (lo * lo) - np.float64(1.0) / (hi * hi)
        a_max = max(a_max, a_s)
    if m == 1 or not a_max > 0.0:
        return int(ndm)
    ratio = a_full / a_max
    g = 1 + int(math.floor(ratio / 2.0))
    return int(min(max(g, 1), ndm))


@dataclass
class Plan:
    freqs: np.ndarray          # [nchan] channel centre frequencies, MHz
    tsamp: float               # sampling time, s
    dms: np.ndarray            # [ndm] fine DM trials, non-decreasing
    nsub: int                  # number of sub-bands
    m: int                     # channels per sub-band
    g: int                     # fine DM trials per coarse group
    ngroups: int               # number of coarse groups, ceil(ndm / g)
    fref: float                # reference frequency = highest channel
    fsub: np.ndarray           # [nsub] sub-band reference = highest channel in it
    coarse_dm: np.ndarray      # [ngroups] coarse DM of each group (its first trial)
    d_coarse_chan: np.ndarray  # [ngroups, nchan] D(c_j, f_ch)
    d_coarse_sub: np.ndarray   # [ngroups, nsub]  D(c_j, f_s)
    d_fine_sub: np.ndarray     # [ndm, nsub]      D(dm_i, f_s)
    extent: np.ndarray         # [ngroups, nsub]  extra stage-1 length of each series
    offsets: np.ndarray        # [ndm, nchan] effective per-channel offset
    overlap: int               # input samples needed beyond the output length

    @property
    def nchan(self):
        return self.freqs.shape[0]

    @property
    def ndm(self):
        return self.dms.shape[0]

    def group_of(self, i):
        return i // self.g


def make_plan(freqs, tsamp, dms, nsub, g=None):
    """Build the two-stage sub-band plan (Sec. 2.3).

    Readings: sub-bands are ``nsub`` equal runs of contiguous channels (nsub
    divides nchan); each sub-band's reference frequency is its highest channel;
    the fine trials are cut into consecutive groups of ``g`` and each group's
    coarse DM is its first (lowest) trial.
    """
    freqs = np.asarray(freqs, dtype=np.float64)
    dms = np.asarray(dms, dtype=np.float64)
    nchan = freqs.shape[0]
    ndm = dms.shape[0]
    if nchan < 1 or ndm < 1 or nsub < 1 or nchan % nsub != 0:
        raise ValueError("bad plan shape")
    if not (np.all(np.isfinite(freqs)) and np.all(freqs > 0)):
        raise ValueError("frequencies must be finite and positive")
    if not (np.all(np.isfinite(dms)) and np.all(dms >= 0) and np.all(np.diff(dms) >= 0)):
        raise ValueError("DM trials must be finite, >= 0 and non-decreasing")
    if not (math.isfinite(tsamp) and tsamp > 0):
        raise ValueError("tsamp must be finite and positive")
    m = nchan // nsub
    if g is None:
        g = group_size_rule(freqs, nsub, ndm)
    g = int(min(max(int(g), 1), ndm))
    ngroups = (ndm + g - 1) // g
    fref = float(np.max(freqs))
    fsub = np.array([np.max(freqs[s * m:(s + 1) * m]) for s in range(nsub)], dtype=np.float64)
    coarse_dm = np.array([dms[j * g] for j in range(ngroups)], dtype=np.float64)

    d_coarse_chan = delay_samples(coarse_dm[:, None], freqs[None, :], fref, tsamp)
    d_coarse_sub = delay_samples(coarse_dm[:, None], fsub[None, :], fref, tsamp)
    d_fine_sub = delay_samples(dms[:, None], fsub[None, :], fref, tsamp)

    group = np.arange(ndm) // g          # group j of each fine trial i
    sub = np.arange(nchan) // m          # sub-band s of each channel ch

    # extent[j, s] = max over i in group j of D(dm_i, f_s) - D(c_j, f_s)
    fine_minus_coarse = d_fine_sub - d_coarse_sub[group, :]          # [ndm, nsub]
    extent = np.zeros((ngroups, nsub), dtype=np.int64)
    for j in range(ngroups):
        extent[j] = np.max(fine_minus_coarse[j * g:min((j + 1) * g, ndm)], axis=0)

    # offsets[i, ch] = D(c_j, f_ch) + D(dm_i, f_s) - D(c_j, f_s)
    offsets = d_coarse_chan[group, :] + fine_minus_coarse[:, sub]

    brute_reach = int(delay_samples(dms[-1], np.min(freqs), fref, tsamp))
    overlap = max(int(offsets.max()), brute_reach)

    return Plan(freqs=freqs, tsamp=float(tsamp), dms=dms, nsub=int(nsub), m=int(m), g=int(g),
                ngroups=int(ngroups), fref=fref, fsub=fsub, coarse_dm=coarse_dm,
                d_coarse_chan=d_coarse_chan, d_coarse_sub=d_coarse_sub, d_fine_sub=d_fine_sub,
                extent=extent, offsets=offsets, overlap=int(overlap))


# ---------------------------------------------------------------------------
# Dedispersion (Sec. 2.3)
# ---------------------------------------------------------------------------

def _acc_dtype(x):
    return np.int64 if np.issubdtype(np.asarray(x).dtype, np.integer) else np.float64


def _check_input(x, nchan, need):
    if x.ndim != 2 or x.shape[0] != nchan or x.shape[1] < need:
        raise ValueError(f"input must be [{nchan}, >= {need}], got {x.shape}")


def channel_rows(x_tf, nchan):
    """The "transpose" step of the dedispersion data flow (Sec. 2.3, Fig.
    "dedispersion_flow"): a block recorded time-major, one row of channel
    samples per time sample, as the channel rows every dedispersion function
    here takes: out[ch][t] = x_tf[t][ch] for ch < nchan."""
    x_tf = np.asarray(x_tf)
    if x_tf.ndim != 2 or x_tf.shape[1] < nchan:
        raise ValueError(f"time-major input must be [nt, >= {nchan}], got {x_tf.shape}")
    return np.ascontiguousarray(x_tf[:, :nchan].T)


def downsample(x, k, nt_out=None):
    """Downsampling in time before dedispersing a DM range (Sec. 2.3, plans
    in DM ranges): each output is the mean of k consecutive samples.  The
    paper does not say how the mean is rounded back to the sample type; the
    reading taken here is to the nearest integer, halves up, i.e.
    (sum + k // 2) // k in integers."""
    x = np.asarray(x)
    if k < 1:
        raise ValueError("k must be >= 1")
    n = x.shape[1] // k if nt_out is None else int(nt_out)
    if n * k > x.shape[1]:
        raise ValueError(f"need {n * k} samples, have {x.shape[1]}")
    s = x[:, :n * k].astype(np.int64).reshape(x.shape[0], n, k).sum(axis=2)
    return ((s + k // 2) // k).astype(x.dtype)


def dedisperse_brute(x, freqs, tsamp, dms, nt):
    """Brute-force dedispersion (Sec. 2.3):
    Y[i][t] = sum over channels of x[ch][t + D(dm_i, f_ch)], t in [0, nt)."""
    freqs = np.asarray(freqs, dtype=np.float64)
    dms = np.asarray(dms, dtype=np.float64)
    fref = float(np.max(freqs))
    d = delay_samples(dms[:, None], freqs[None, :], fref, tsamp)
    _check_input(x, freqs.shape[0], nt + (int(d.max()) if d.size else 0))
    y = np.zeros((dms.shape[0], nt), dtype=_acc_dtype(x))
    for i in range(dms.shape[0]):
        for ch in range(freqs.shape[0]):
            y[i] += x[ch, d[i, ch]:d[i, ch] + nt]
    return y


def subband_stage1(x, plan: Plan, nt):
    """First stage (Sec. 2.3, step 1 of the sub-band method): dedisperse every
    sub-band at each coarse DM.  Returns ``B[j][s]``, a series of length
    nt + extent[j, s]:  B[j][s][u] = sum over ch in s of x[ch][u + D(c_j, f_ch)].
    The extra length lets the second stage shift each series by up to the
    largest fine-minus-coarse sub-band delay in the group."""
    _check_input(x, plan.nchan, nt + plan.overlap)
    out = []
    for j in range(plan.ngroups):
        row = []
        for s in range(plan.nsub):
            n = nt + int(plan.extent[j, s])
            acc = np.zeros(n, dtype=_acc_dtype(x))
            for ch in range(s * plan.m, (s + 1) * plan.m):
                d = int(plan.d_coarse_chan[j, ch])
                acc += x[ch, d:d + n]
            row.append(acc)
        out.append(row)
    return out


def subband_stage2(B, plan: Plan, nt):
    """Second stage (Sec. 2.3, step 3 of the sub-band method): dedisperse the
    sub-banded series on the fine grid.
    Y[i][t] = sum over s of B[j][s][t + D(dm_i, f_s) - D(c_j, f_s)], j = group of i.
    (The paper's DM/frequency transpose between the stages is a memory-layout
    step and changes no value.)"""
    dtype = B[0][0].dtype
    y = np.zeros((plan.ndm, nt), dtype=dtype)
    for i in range(plan.ndm):
        j = plan.group_of(i)
        for s in range(plan.nsub):
            e = int(plan.d_fine_sub[i, s] - plan.d_coarse_sub[j, s])
            y[i] += B[j][s][e:e + nt]
    return y


def dedisperse_subband(x, plan: Plan, nt):
    """Two-stage sub-band dedispersion: stage 1 then stage 2."""
    return subband_stage2(subband_stage1(x, plan, nt), plan, nt)


def dedisperse_offsets(x, offsets, nt):
    """One-stage sum with a per-(trial, channel) offset table:
    Y[i][t] = sum over ch of x[ch][t + offsets[i, ch]].  With the plan's
    effective offsets this is the same sum the two stages compute; with the
    brute-force delay table it is brute force."""
    offsets = np.asarray(offsets, dtype=np.int64)
    ndm, nchan = offsets.shape
    _check_input(x, nchan, nt + (int(offsets.max()) if offsets.size else 0))
    y = np.zeros((ndm, nt), dtype=_acc_dtype(x))
    for i in range(ndm):
        for ch in range(nchan):
            o = int(offsets[i, ch])
            y[i] += x[ch, o:o + nt]
    return y


# ---------------------------------------------------------------------------
# Matched filter (Sec. 2.4, Eq. 5) and the DM-time plane (Sec. 2.5)
# ---------------------------------------------------------------------------

@dataclass
class DMStats:
    sum_y: int      # exact sum of the series
    c: int          # floor(sum_y / T)
    q: int          # exact sum of (y - c)^2
    r: int          # sum_y - T * c
    var: float      # population variance of the block
    sigma: float    # sqrt(var)
    inv_d: float    # 1 / (sigma * T)


def dm_stats(y):
    """Noise statistics of one dedispersed series (the sigma of Sec. 2.4, Eq. 5).

    Reading: sigma is the population standard deviation of the block's T
    samples, from exact integer sums: c = floor(sum/T), Q = sum (y - c)^2,
    r = sum - T c, var = Q/T - (r/T)^2, all float64 in this order."""
    y = np.asarray(y)
    T = int(y.shape[0])
    v = y.astype(np.int64)
    sum_y = int(np.sum(v))              # exact: |y| < 2^21, T <= 2^21
    c = sum_y // T
    q = int(np.sum((v - c) * (v - c)))  # exact in int64 under the same bounds
    r = sum_y - T * c
    a = float(q) / float(T)
    b = float(r) / float(T)
    var = a - b * b
    if var > 0.0:
        sigma = math.sqrt(var)
        inv_d = 1.0 / (sigma * float(T))
    else:
        sigma = 0.0
        inv_d = 0.0
    return DMStats(sum_y=sum_y, c=c, q=q, r=r, var=var, sigma=sigma, inv_d=inv_d)


def snr_from_sum(S, w, T, sum_y, inv_d):
    """Boxcar S/N of a window of width ``w`` whose exact sum is ``S``
    (Sec. 2.4, Eq. 5 with the block mean removed):
    S/N = (S - w * mean) / (sigma * sqrt(w)) = N / (T sigma) / sqrt(w),
    N = T S - w sum_y, evaluated as ((double) N * inv_d) * (1 / sqrt(w))."""
    N = int(T) * int(S) - int(w) * int(sum_y)
    rsw = 1.0 / math.sqrt(float(w))
    return (float(N) * inv_d) * rsw


def _prefix(y):
    """Running sum P[t] = sum_{k < t} y[k], t in [0, T] (step (1) of Sec. 2.4)."""
    p = np.zeros(y.shape[0] + 1, dtype=np.int64)
    np.cumsum(y.astype(np.int64), out=p[1:])
    return p


def _window_sums(p, w):
    """Sums of the windows [t, t + w), t in [0, T - w]: the difference of two
    running-sum values (step (2) of Sec. 2.4).  Reading of the window: it
    starts at t and holds exactly w samples; only windows inside the block."""
    T = p.shape[0] - 1
    return p[w:T + 1] - p[0:T - w + 1]


def boxcar_snr_series(y, w):
    """S/N of every window of width ``w`` in one series (t in [0, T - w]),
    evaluated exactly as ``snr_from_sum`` does."""
    y = np.asarray(y)
    T = int(y.shape[0])
    st = dm_stats(y)
    if not st.var > 0.0 or w > T:
        return np.zeros(max(T - w + 1, 0))
    S = _window_sums(_prefix(y), w)
    N = (np.int64(T) * S - np.int64(w) * np.int64(st.sum_y)).astype(np.float64)
    return (N * st.inv_d) * (1.0 / math.sqrt(float(w)))


def boxcar_peak(y, widths):
    """Peak boxcar S/N of one series: returns (snr, width, start time).

    For each width the earliest start maximising the exact window sum is
    taken; the width with the largest S/N wins and ties go to the smaller
    width.  Widths longer than the block are skipped.  A block with zero
    variance (or no usable width) gives (0.0, widths[0], 0)."""
    y = np.asarray(y)
    T = int(y.shape[0])
    st = dm_stats(y)
    if not st.var > 0.0:
        return (0.0, int(widths[0]), 0)
    p = _prefix(y)
    best = None
    for w in sorted(int(v) for v in widths):
        if w > T:
            continue
        S = _window_sums(p, w)
        t = int(np.argmax(S))
        snr = snr_from_sum(int(S[t]), w, T, st.sum_y, st.inv_d)
        if best is None or snr > best[0]:
            best = (snr, w, t)
    if best is None:
        return (0.0, int(widths[0]), 0)
    return best


def boxcar_peaks(Y, widths):
    """``boxcar_peak`` for every row of a DM x time array."""
    out = [boxcar_peak(Y[i], widths) for i in range(Y.shape[0])]
    snr = np.array([o[0] for o in out], dtype=np.float64)
    wid = np.array([o[1] for o in out], dtype=np.int32)
    tim = np.array([o[2] for o in out], dtype=np.int64)
    return snr, wid, tim


def boxcar_candidates(Y, widths, gamma, dm_offset=0):
    """Thresholded DM-time plane (Sec. 2.5): for each (DM row d, start t),
    the width with the highest S/N (ties to the smaller width); the point is
    kept when that S/N is at least ``gamma``.  Returns a list of
    (d, t, width, snr) sorted by (d, t).  Rows with zero variance give none."""
    widths = sorted(int(v) for v in widths)
    out = []
    for d in range(Y.shape[0]):
        y = np.asarray(Y[d])
        T = int(y.shape[0])
        st = dm_stats(y)
        if not st.var > 0.0:
            continue
        p = _prefix(y)
        grid = np.full((len(widths), T), -np.inf, dtype=np.float64)
        for k, w in enumerate(widths):
            if w > T:
                continue
            S = _window_sums(p, w)
            N = (np.int64(T) * S - np.int64(w) * np.int64(st.sum_y)).astype(np.float64)
            rsw = 1.0 / math.sqrt(float(w))
            grid[k, :T - w + 1] = (N * st.inv_d) * rsw
        kbest = np.argmax(grid, axis=0)
        sbest = grid[kbest, np.arange(T)]
        for t in np.nonzero(sbest >= gamma)[0]:
            out.append((d + dm_offset, int(t), widths[int(kbest[t])], float(sbest[t])))
    return out


def boxcar_snr_fixed(y, widths, mean, sigma):
    """Boxcar S/N with a given noise mean and sigma (no estimation):
    max over t of (S_w(t) - w * mean) / (sigma * sqrt(w)) for each width.
    Used to check Eq. 5 and the width-mismatch loss of Sec. 2.4 on
    noise-free pulses."""
    y = np.asarray(y, dtype=np.float64)
    T = y.shape[0]
    p = np.zeros(T + 1, dtype=np.float64)
    np.cumsum(y, out=p[1:])
    out = []
    for w in widths:
        S = p[w:T + 1] - p[0:T - w + 1]
        out.append(float(np.max((S - w * mean) / (sigma * math.sqrt(w)))))
    return np.array(out)


# ---------------------------------------------------------------------------
# Clustering of the DM-time plane (Sec. 2.5)
# ---------------------------------------------------------------------------

def delay_axis(dms, freqs, tsamp):
    """DM turned into dispersion delay (Sec. 2.5 uses Eq. 1 so that both axes
    of the DM-time plane are times).  Reading: the delay across the band, from
    the highest to the lowest channel frequency, in samples and unrounded,
    ((k DM) (1/f_lo^2 - 1/f_hi^2)) / tsamp in float64 in this order."""
    freqs = np.asarray(freqs, dtype=np.float64)
    f_lo, f_hi = np.float64(freqs.min()), np.float64(freqs.max())
    inv = np.float64(1.0) / (f_lo * f_lo) - np.float64(1.0) / (f_hi * f_hi)
    return ((np.float64(K_DM) * np.asarray(dms, dtype=np.float64)) * inv) / np.float64(tsamp)


def dbscan_plane(points, dms, freqs, tsamp, radius, min_pts):
    """DBSCAN (Sec. 2.5) of DM-time points ``points`` = [(d, t, w, snr), ...]
    (d a DM trial index, t a start sample), by the definitions the paper gives:

    * neighbours of p: the other points within Euclidean distance ``radius``
      in the (delay, time) plane, both in samples;
    * core point: more than ``min_pts`` neighbours (the paper's "exceeds");
    * a cluster: all core points joined by chains of core neighbours, plus the
      non-core points within ``radius`` of them ("reachable" points);
    * everything else is noise.

    Readings where the paper leaves a choice: a non-core point within reach of
    several clusters joins the one of its nearest core neighbour (ties: the
    first in (d, t) order); points are ordered by (d, t), clusters numbered by
    their first core point; a cluster's representative (the candidate that
    survives de-duplication) is its highest-S/N point, ties to the first.

    Returns (sorted points, labels (-1 noise), representatives (sorted index
    per cluster), number of clusters).  Plain O(n^2) pairwise distances.
    """
    pts = sorted((int(d), int(t), int(w), float(snr)) for d, t, w, snr in points)
    n = len(pts)
    xs = delay_axis(dms, freqs, tsamp)
    x = np.array([xs[d] for d, _, _, _ in pts], dtype=np.float64)
    t = np.array([tt for _, tt, _, _ in pts], dtype=np.float64)
    r2 = np.float64(radius) * np.float64(radius)
    nbr = []
    dist2 = []
    for i in range(n):
        dx = x - x[i]
        dt = t - t[i]
        d2 = dx * dx + dt * dt
        mask = d2 <= r2
        mask[i] = False
        nbr.append(np.nonzero(mask)[0])
        dist2.append(d2)
    core = np.array([len(nb) > min_pts for nb in nbr], dtype=bool)
    # connected components of the core graph (breadth-first), root = smallest index
    comp = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        if not core[i] or comp[i] >= 0:
            continue
        comp[i] = i
        queue = [i]
        while queue:
            a = queue.pop()
            for b in nbr[a]:
                if core[b] and comp[b] < 0:
                    comp[b] = i
                    queue.append(b)
    root = comp.copy()
    for i in range(n):
        if core[i]:
            continue
        best = None
        for q in nbr[i]:
            if core[q] and (best is None or dist2[i][q] < dist2[i][best] or (dist2[i][q] == dist2[i][best] and q < best)):
                best = q
        root[i] = comp[best] if best is not None else -1
    roots = sorted(set(int(r) for r in root[core]))
    cid = {r: c for c, r in enumerate(roots)}
    labels = np.array([cid[int(r)] if r >= 0 else -1 for r in root], dtype=np.int64)
    reps = []
    for c in range(len(roots)):
        members = [i for i in range(n) if labels[i] == c]
        reps.append(max(members, key=lambda i: (pts[i][3], -i)))
    return pts, labels, np.array(reps, dtype=np.int64), len(roots)


# ---------------------------------------------------------------------------
# Narrow-band RFI: channel statistics and mask (Sec. 2.2)
# ---------------------------------------------------------------------------

def channel_power_sums(x):
    """Per channel row: (sum x, sum x^2, sum x^3, sum x^4), exact integers."""
    x = np.asarray(x).astype(np.int64)
    return np.stack([(x ** j).sum(axis=1) for j in (1, 2, 3, 4)], axis=1)


def channel_moments(sums, nt):
    """Skewness m3 / m2^1.5 and kurtosis m4 / m2^2 of each channel from its
    power sums over nt samples (population central moments).  The central
    moments are formed exactly in integers (n^2 m2, n^3 m3, n^4 m4) and turned
    to float64 once; channels with m2 = 0 give None."""
    out = []
    n = int(nt)
    for s1, s2, s3, s4 in np.asarray(sums).tolist():
        s1, s2, s3, s4 = int(s1), int(s2), int(s3), int(s4)
        m2 = n * s2 - s1 * s1
        m3 = n * n * s3 - 3 * n * s1 * s2 + 2 * s1 ** 3
        m4 = n ** 3 * s4 - 4 * n * n * s1 * s3 + 6 * n * s1 * s1 * s2 - 3 * s1 ** 4
        if m2 <= 0:
            out.append(None)
            continue
        f2, f3, f4 = float(m2), float(m3), float(m4)
        out.append((f3 / (f2 * np.sqrt(f2)), f4 / (f2 * f2)))
    return out


def skf_mask(sums, nt, threshold):
    """The skewness-kurtosis filter (Sec. 2.2): channels that are outliers in
    skewness or kurtosis across the band are removed.  The paper states the
    intent; the rule taken here (a reading) is the robust z-score: over the
    channels with non-zero variance, a value s is an outlier when
    |s - median| > threshold * 1.482602218505602 * MAD (MAD the median absolute
    deviation; with MAD = 0, any value off the median).  Returns uint8, 0 for
    removed channels (outliers, and channels of zero variance), 1 to keep."""
    mom = channel_moments(sums, nt)
    idx = [c for c, m in enumerate(mom) if m is not None]
    mask = np.zeros(len(mom), dtype=np.uint8)
    if not idx:
        return mask

    def med(v):
        v = sorted(v)
        k = len(v)
        return v[k // 2] if k % 2 else (v[k // 2 - 1] + v[k // 2]) / 2.0

    bad = [False] * len(idx)
    for j in (0, 1):
        s = [mom[c][j] for c in idx]
        m = med(s)
        dev = [abs(v - m) for v in s]
        mad = med(dev)
        lim = threshold * (1.482602218505602 * mad)
        for i, dv in enumerate(dev):
            bad[i] = bad[i] or (dv > lim if mad > 0.0 else dv != 0.0)
    for i, c in enumerate(idx):
        mask[c] = 0 if bad[i] else 1
    return mask



# ---------------------------------------------------------------------------
# Normalisation (Sec. 2.1) and dedispersion of normalised data
# ---------------------------------------------------------------------------

WEIGHT_UNIT = 0          # scale a channel by 1 / sigma: zero mean, unit variance
WEIGHT_INVERSE_VAR = 1   # scale a channel by 1 / sigma^2: each channel weighted by its inverse variance


def channel_mean_var(sums, nt):
    """Mean and population variance of each channel from its exact sums
    (sum x, sum x^2, ...) over nt samples: mean = S1 / n and
    var = (n S2 - S1^2) / n^2, the numerator an exact integer, each turned
    to float64 once."""
    n = int(nt)
    out = []
    for row in np.asarray(sums).tolist():
        s1, s2 = int(row[0]), int(row[1])
        out.append((float(s1) / float(n), float(n * s2 - s1 * s1) / float(n * n)))
    return out


def norm_weights(sums, nt, weighting=WEIGHT_UNIT):
    """Per-channel normalisation of Sec. 2.1 as (scale, offset) pairs, so
    that a channel's normalised sample is scale * x - offset:
      * WEIGHT_UNIT: scale = 1 / sigma, offset = mean / sigma (mean zero and
        unit variance in every channel; the paper's "adjusting the data to a
        mean of zero and unity variance");
      * WEIGHT_INVERSE_VAR: scale = 1 / sigma^2, offset = mean / sigma^2 (the
        reading of its "reweighting ... with the reciprocal of its variance"
        as inverse-variance weights).
    A channel of zero variance gets (0, 0): it adds nothing.  Computed in
    float64 and rounded to float32 once (the values both the oracle and the
    device kernels then use), returned as float64 arrays holding those
    float32 values."""
    scale = np.zeros(len(sums), dtype=np.float64)
    offset = np.zeros(len(sums), dtype=np.float64)
    for c, (mean, var) in enumerate(channel_mean_var(sums, nt)):
        if not var > 0.0:
            continue
        s = 1.0 / math.sqrt(var) if weighting == WEIGHT_UNIT else 1.0 / var
        scale[c] = float(np.float32(s))
        offset[c] = float(np.float32(s * mean))
    return scale, offset


def normalise(x, scale, offset):
    """The normalised block: scale[c] * x[c][t] - offset[c], float64 (exact
    for float32 scale and offset and uint8 samples but for one rounding)."""
    x = np.asarray(x).astype(np.float64)
    return x * np.asarray(scale, dtype=np.float64)[:, None] - np.asarray(offset, dtype=np.float64)[:, None]


def dedisperse_subband_norm(x, plan: Plan, nt, scale, offset):
    """Two-stage sub-band dedispersion (Sec. 2.3) of the normalised block,
    in float64: stage 1 at the coarse DMs per sub-band, stage 2 at the fine
    DMs, the same plan and offsets as the integer path."""
    return dedisperse_subband(normalise(x, scale, offset), plan, nt)


def norm_abs_bound(x, plan: Plan, nt, scale, offset):
    """Per output, the sum over channels of |normalised sample| it adds:
    sum_ch |scale x - offset| at the sample's effective offset.  A float32
    evaluation that rounds every channel term once and sums m terms per
    sub-band then nsub per trial errs by at most (m + nsub + 1) 2^-24 times
    this (the recursive-summation bound); the tests use it as the tolerance."""
    a = np.abs(normalise(x, scale, offset))
    return dedisperse_offsets(a, plan.offsets, nt)


def float_stats(y):
    """Noise statistics of one float series for the matched filter: the
    population mean and variance of its T values, from their float64 sums,
    var = S2 / T - (S1 / T)^2.  Returns (mean, var)."""
    y = np.asarray(y, dtype=np.float64)
    T = float(y.shape[0])
    s1 = float(np.sum(y))
    s2 = float(np.sum(y * y))
    mean = s1 / T
    return mean, s2 / T - mean * mean


def boxcar_snr_series_float(y, w):
    """S/N of every window [t, t + w) of a float series (Sec. 2.4, Eq. 5):
    (S - w mean) / (sigma sqrt(w)), S from a float64 running sum."""
    y = np.asarray(y, dtype=np.float64)
    T = y.shape[0]
    mean, var = float_stats(y)
    if not var > 0.0 or w > T:
        return np.zeros(max(T - w + 1, 0))
    p = np.zeros(T + 1, dtype=np.float64)
    np.cumsum(y, out=p[1:])
    S = p[w:T + 1] - p[0:T - w + 1]
    return (S - w * mean) / (math.sqrt(var) * math.sqrt(float(w)))


def boxcar_peaks_float(Y, widths):
    """Per row: (snr, width, start) of the largest S/N over widths and
    starts (per width the earliest start with the largest window sum; ties
    across widths to the smaller width); (0, widths[0], 0) for a row of zero
    variance."""
    widths = sorted(int(v) for v in widths)
    out = []
    for d in range(Y.shape[0]):
        y = np.asarray(Y[d], dtype=np.float64)
        mean, var = float_stats(y)
        best = None
        if var > 0.0:
            for w in widths:
                if w > y.shape[0]:
                    continue
                s = boxcar_snr_series_float(y, w)
                t = int(np.argmax(s))
                if best is None or s[t] > best[0]:
                    best = (float(s[t]), w, t)
        out.append(best if best is not None else (0.0, widths[0], 0))
    return (np.array([o[0] for o in out]), np.array([o[1] for o in out], dtype=np.int32),
            np.array([o[2] for o in out], dtype=np.int64))


def boxcar_candidates_float(Y, widths, gamma):
    """The thresholded DM-time plane (Sec. 2.5) of float series: (d, t,
    width, snr) for every start whose best width (ties to the smaller) has
    S/N >= gamma, sorted by (d, t)."""
    widths = sorted(int(v) for v in widths)
    out = []
    for d in range(Y.shape[0]):
        y = np.asarray(Y[d], dtype=np.float64)
        T = y.shape[0]
        _, var = float_stats(y)
        if not var > 0.0:
            continue
        grid = np.full((len(widths), T), -np.inf)
        for k, w in enumerate(widths):
            if w <= T:
                grid[k, :T - w + 1] = boxcar_snr_series_float(y, w)
        kb = np.argmax(grid, axis=0)
        sb = grid[kb, np.arange(T)]
        for t in np.nonzero(sb >= gamma)[0]:
            out.append((d, int(t), widths[int(kb[t])], float(sb[t])))
    return out
