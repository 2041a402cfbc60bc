"""Autotuning of the plan shape: tile variants per plan (measured by
``tx_plan_autotune`` on the device) and the sub-band count, with a JSON cache
so that a shape is measured once per device.

Tiles and the sub-band count change only speed and scratch size: the tile
choice never changes the output, and every sub-band count gives the exact
two-stage result for that count (the plan reports it, with the DMs-per-group
that the smearing rule derives from it).  The DMs-per-group itself is not
tuned: it sets the accuracy of the approximation (Sec. 2.3), not its speed
alone.
"""

import hashlib
import json
import os

import numpy as np

import paper_2401_13834_amd as tx

_ENV = "TX_TUNE_CACHE"


def cache_path():
    """``$TX_TUNE_CACHE``, else ``~/.cache/paper_2401_13834_amd/tiles.json``."""
    p = os.environ.get(_ENV)
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2401_13834_amd", "tiles.json")


def _digest(freqs, tsamp, dms):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(freqs, dtype=np.float64).tobytes())
    h.update(np.float64(tsamp).tobytes())
    h.update(np.ascontiguousarray(dms, dtype=np.float64).tobytes())
    return h.hexdigest()[:20]


def shape_key(freqs, tsamp, dms, nsub, nt, device):
    """Cache key of a plan shape, block length and device name."""
    return f"{device}|{_digest(freqs, tsamp, dms)}|nsub={int(nsub)}|nt={int(nt)}"


def load(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save(entries, path=None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _device_name():
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device()).replace("|", "/")


def tune_tiles(plan, freqs, tsamp, dms, nt, *, effort=1, path=None, refresh=False):
    """Set ``plan``'s tiles from the cache, or measure and cache them.
    Returns ((stage1, stage1_lds, stage2, stage2_lds), milliseconds per
    dedispersion, or None when the cache answered)."""
    key = shape_key(freqs, tsamp, dms, plan.nsub, nt, _device_name())
    entries = load(path)
    ent = entries.get(key)
    if ent and not refresh:
        plan.set_tiles(*ent["tiles"])
        return tuple(ent["tiles"]), None
    ms = plan.autotune(nt, effort=effort)
    tiles = plan.get_tiles()
    entries = load(path)
    entries[key] = {"tiles": list(tiles), "ms": ms}
    save(entries, path)
    return tiles, ms


def nsub_candidates(nchan, max_m=256):
    """Sub-band counts that divide the channel count with at most ``max_m``
    channels per sub-band (the first stage sums at most 256 bytes per 16-bit
    lane)."""
    return [d for d in range(1, nchan + 1) if nchan % d == 0 and nchan // d <= max_m]


def plan_autotuned(freqs, tsamp, dms, nt, *, nsubs=None, effort=1, path=None, refresh=False):
    """The fastest plan over sub-band counts ``nsubs`` (default: the divisors
    within a factor of four of the library's cost-model choice), each with
    tuned tiles.  Returns (plan, {nsub: ms})."""
    base = tx.tx_plan(freqs, tsamp, dms, 0)
    if nsubs is None:
        c = base.nsub
        nsubs = [d for d in nsub_candidates(len(freqs)) if c / 4 <= d <= 4 * c]
    key = shape_key(freqs, tsamp, dms, 0, nt, _device_name()) + "|nsub-search"
    entries = load(path)
    ent = entries.get(key)
    if ent and not refresh and int(ent["nsub"]) in nsubs:
        plan = tx.tx_plan(freqs, tsamp, dms, int(ent["nsub"]))
        tune_tiles(plan, freqs, tsamp, dms, nt, effort=effort, path=path)
        return plan, {int(k): v for k, v in ent["ms"].items()}
    times = {}
    best = None
    for ns in nsubs:
        plan = tx.tx_plan(freqs, tsamp, dms, int(ns))
        _, ms = tune_tiles(plan, freqs, tsamp, dms, nt, effort=effort, path=path, refresh=True)
        times[int(ns)] = ms
        if best is None or ms < times[best.nsub]:
            best = plan
    entries = load(path)
    entries[key] = {"nsub": best.nsub, "ms": {str(k): v for k, v in times.items()}}
    save(entries, path)
    return best, times
