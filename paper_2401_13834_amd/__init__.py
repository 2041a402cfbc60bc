"""Python binding of libtx (include/tx.h): argument marshalling only.

Every computation runs in the HIP library ``libtx.so`` built in this
directory (``python -m paper_2401_13834_amd.build``).  If the library is not
built, importing the binding's functions raises; there is no fallback.

Device buffers are passed as torch tensors (only their ``data_ptr()`` and
shape are used); streams are torch streams or raw ``hipStream_t`` integers.
The names mirror the C entry points.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtx.so")

TX_OK, TX_EINVAL, TX_ENOMEM, TX_EDEVICE, TX_ESTATE, TX_EOVERFLOW, TX_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
STATUS = {0: "TX_OK", -1: "TX_EINVAL", -2: "TX_ENOMEM", -3: "TX_EDEVICE", -4: "TX_ESTATE",
          -5: "TX_EOVERFLOW", -6: "TX_ENOTSUP"}
TX_PLAN_HOST_ONLY = 1
TX_MAX_WIDTHS = 32

CAND_DTYPE = np.dtype([("dm_index", "<i4"), ("width", "<i4"), ("time", "<i8"), ("snr", "<f8")])

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_dblp = ctypes.POINTER(ctypes.c_double)


class TxError(RuntimeError):
    def __init__(self, status, what):
        detail = ""
        if status in (-2, -3, -6) and _lib is not None:
            detail = " (" + (_lib.tx_last_error() or b"").decode() + ")"
        super().__init__(f"{what}: {STATUS.get(status, status)}{detail}")
        self.status = status


class Tiles(ctypes.Structure):
    """tx_tiles: kernel variant and LDS bytes per workgroup of each stage (-1 / 0 = defaults)."""
    _fields_ = [("stage1", ctypes.c_int32), ("stage1_lds", ctypes.c_int32), ("stage2", ctypes.c_int32),
                ("stage2_lds", ctypes.c_int32)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("nchan", ctypes.c_int32), ("ndm", ctypes.c_int32), ("nsub", ctypes.c_int32),
                ("chans_per_sub", ctypes.c_int32), ("g", ctypes.c_int32), ("ngroups", ctypes.c_int32),
                ("overlap", ctypes.c_int64), ("max_extent", ctypes.c_int64), ("brute_reach", ctypes.c_int64),
                ("fref_mhz", ctypes.c_double), ("tsamp_s", ctypes.c_double), ("on_device", ctypes.c_int32),
                ("device", ctypes.c_int32)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "tx_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "tx_version": (ctypes.c_char_p, []),
    "tx_last_error": (ctypes.c_char_p, []),
    "tx_plan": (ctypes.c_int, [_c_dblp, ctypes.c_int32, ctypes.c_double, _c_dblp, ctypes.c_int32, ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_void_p)]),
    "tx_plan_ex": (ctypes.c_int, [_c_dblp, ctypes.c_int32, ctypes.c_double, _c_dblp, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]),
    "tx_plan_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_PlanInfo)]),
    "tx_plan_offsets": (ctypes.c_int, [ctypes.c_void_p, _c_i32p]),
    "tx_plan_tables": (ctypes.c_int, [ctypes.c_void_p, _c_i32p, _c_i32p, _c_i32p, _c_i32p]),
    "tx_plan_delays": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, _c_i32p]),
    "tx_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "tx_dedisperse_ws_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "tx_dedisperse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "tx_dedisperse_ws": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p]),
    "tx_dedisperse_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "tx_boxcar_snr": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _c_i32p,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "tx_candidates": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _c_i32p,
                                     ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "tx_tile_variants": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "tx_tile_variant_info": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "tx_plan_get_tiles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tx_plan_resolved_tiles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "tx_plan_set_tiles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tx_profile_enable": (ctypes.c_int, [ctypes.c_int32]),
    "tx_profile_collect": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64)]),
}

TX_KERNEL_STAGE1, TX_KERNEL_STAGE2, TX_KERNEL_BOXCAR, TX_KERNEL_TRANSPOSE, TX_KERNEL_DOWNSAMPLE = 0, 1, 2, 3, 4


def lib():
    """The loaded libtx (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2401_13834_amd.build`")
        # torch ships its own HIP runtime under the same soname.  Load it first
        # so that libtx binds to that one runtime: torch's streams and device
        # memory are then valid in libtx, and only one runtime owns the GPU.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return list(_SIGS)


def _check(status, what):
    if status != TX_OK:
        raise TxError(status, what)


def _dbl(arr):
    a = np.ascontiguousarray(arr, dtype=np.float64)
    return a, a.ctypes.data_as(_c_dblp)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, name):
    """Argument check: ``t`` is a tensor of ``dtype`` ("uint8", "int32", ...)
    whose rows, if it has two dimensions, are contiguous (the library takes a
    base pointer and a row pitch in elements of that type)."""
    if t is None:
        return t
    if str(t.dtype) != "torch." + dtype:
        raise TypeError(f"{name}: a {dtype} tensor is expected, not {t.dtype}")
    if t.dim() == 2 and t.numel() > 0 and t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name}: the rows of the tensor must be contiguous")
    return t


def _need_peaks(peaks, name):
    if peaks is not None:
        _need(peaks[0], "float64", name + " snr")
        _need(peaks[1], "int32", name + " width")
        _need(peaks[2], "int64", name + " time")
    return peaks


class Plan:
    """Owner of a ``tx_plan_t``."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)
        info = _PlanInfo()
        _check(lib().tx_plan_query(self._h, ctypes.byref(info)), "tx_plan_query")
        self.info = {f: getattr(info, f) for f, _ in _PlanInfo._fields_}

    @property
    def handle(self):
        return self._h

    def __getattr__(self, name):
        info = self.__dict__.get("info")
        if info is not None and name in info:
            return info[name]
        raise AttributeError(name)

    def offsets(self):
        out = np.empty((self.info["ndm"], self.info["nchan"]), dtype=np.int32)
        _check(lib().tx_plan_offsets(self._h, out.ctypes.data_as(_c_i32p)), "tx_plan_offsets")
        return out

    def tables(self):
        i = self.info
        cc = np.empty((i["ngroups"], i["nchan"]), dtype=np.int32)
        cs = np.empty((i["ngroups"], i["nsub"]), dtype=np.int32)
        fs = np.empty((i["ndm"], i["nsub"]), dtype=np.int32)
        ex = np.empty((i["ngroups"], i["nsub"]), dtype=np.int32)
        _check(lib().tx_plan_tables(self._h, *(a.ctypes.data_as(_c_i32p) for a in (cc, cs, fs, ex))),
               "tx_plan_tables")
        return {"coarse_chan": cc, "coarse_sub": cs, "fine_sub": fs, "extent": ex}

    def delays(self, dm):
        out = np.empty(self.info["nchan"], dtype=np.int32)
        _check(lib().tx_plan_delays(self._h, float(dm), out.ctypes.data_as(_c_i32p)), "tx_plan_delays")
        return out

    def set_mask(self, mask):
        """mask: nchan values, 0 drops a channel from every sum (None keeps all)."""
        if mask is None:
            _check(lib().tx_plan_set_mask(self._h, None), "tx_plan_set_mask")
            return
        m = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8)
        if m.size != self.info["nchan"]:
            raise ValueError("mask needs one value per channel")
        _check(lib().tx_plan_set_mask(self._h, m.ctypes.data_as(ctypes.c_void_p)), "tx_plan_set_mask")

    def get_mask(self):
        m = np.empty(self.info["nchan"], dtype=np.uint8)
        _check(lib().tx_plan_get_mask(self._h, m.ctypes.data_as(ctypes.c_void_p)), "tx_plan_get_mask")
        return m

    def get_tiles(self):
        t = Tiles()
        _check(lib().tx_plan_get_tiles(self._h, ctypes.byref(t)), "tx_plan_get_tiles")
        return (t.stage1, t.stage1_lds, t.stage2, t.stage2_lds)

    def resolved_tiles(self, nt):
        """(stage1, stage1_lds, stage2, stage2_lds) a dedispersion of ``nt``
        outputs launches with, defaults resolved."""
        t = Tiles()
        _check(lib().tx_plan_resolved_tiles(self._h, int(nt), ctypes.byref(t)), "tx_plan_resolved_tiles")
        return (t.stage1, t.stage1_lds, t.stage2, t.stage2_lds)

    def set_tiles(self, stage1=-1, stage1_lds=0, stage2=-1, stage2_lds=0):
        t = Tiles(stage1, stage1_lds, stage2, stage2_lds)
        _check(lib().tx_plan_set_tiles(self._h, ctypes.byref(t)), "tx_plan_set_tiles")

    def autotune(self, nt, effort=1, stream=None):
        """Measure the tile variants for blocks of ``nt`` outputs on the current
        device and keep the fastest; returns its time in milliseconds."""
        ms = ctypes.c_double()
        _check(_setup_more().tx_plan_autotune(self._h, int(nt), int(effort), ctypes.byref(ms), _stream(stream)),
               "tx_plan_autotune")
        return ms.value

    def ws_size(self, nt):
        b = ctypes.c_int64()
        _check(lib().tx_dedisperse_ws_size(self._h, int(nt), ctypes.byref(b)), "tx_dedisperse_ws_size")
        return b.value

    def close(self):
        if self._h is not None and self._h.value:
            lib().tx_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tx_plan(freqs_mhz, tsamp_s, dms, nsub, *, dms_per_group=0, host_only=False):
    f, fp = _dbl(freqs_mhz)
    d, dp = _dbl(dms)
    h = ctypes.c_void_p()
    flags = TX_PLAN_HOST_ONLY if host_only else 0
    _check(lib().tx_plan_ex(fp, len(f), float(tsamp_s), dp, len(d), int(nsub), int(dms_per_group), flags,
                            ctypes.byref(h)), "tx_plan")
    return Plan(h.value)


def tx_dedisperse(plan, d_in, nt, d_out, stream=None, ws=None):
    """d_in: uint8 device tensor [nchan, in_pitch]; d_out: int32 [ndm, out_pitch]."""
    _need(d_in, "uint8", "tx_dedisperse d_in")
    _need(d_out, "int32", "tx_dedisperse d_out")
    in_pitch = d_in.stride(0) * d_in.element_size()
    out_pitch = d_out.stride(0)
    if ws is None:
        st = lib().tx_dedisperse(plan.handle, _ptr(d_in), in_pitch, int(nt), _ptr(d_out), out_pitch,
                                 _stream(stream))
    else:
        st = lib().tx_dedisperse_ws(plan.handle, _ptr(d_in), in_pitch, int(nt), _ptr(d_out), out_pitch,
                                    _ptr(ws), ws.numel() * ws.element_size(), _stream(stream))
    _check(st, "tx_dedisperse")


TX_WEIGHT_UNIT, TX_WEIGHT_INVERSE_VAR = 0, 1

_SIGS3 = {
    "tx_norm_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "tx_dedisperse_norm": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p]),
    "tx_dedisperse_norm_ws_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "tx_boxcar_snr_f32": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _c_i32p,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "tx_boxcar_snr_fixed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _c_i32p,
                                           ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tx_candidates_f32": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _c_i32p,
                                         ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
}
_SIGS.update(_SIGS3)


def _setup_norm():
    L = lib()
    for name, (res, args) in _SIGS3.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def tx_norm_weights(sums, nt, weighting=TX_WEIGHT_UNIT):
    """Per-channel (scale, offset) float32 arrays from power sums [nchan, 4] (host)."""
    s = np.ascontiguousarray(sums, dtype=np.uint64)
    nchan = s.shape[0]
    scale = np.empty(nchan, dtype=np.float32)
    offset = np.empty(nchan, dtype=np.float32)
    _check(_setup_norm().tx_norm_weights(s.ctypes.data, nchan, int(nt), int(weighting), scale.ctypes.data,
                                         offset.ctypes.data), "tx_norm_weights")
    return scale, offset


def tx_dedisperse_norm(plan, d_in, nt, d_scale, d_offset, d_out, stream=None):
    """d_in uint8 [nchan, pitch]; d_scale, d_offset float32 [nchan]; d_out float32 [ndm, pitch]."""
    _need(d_in, "uint8", "tx_dedisperse_norm d_in")
    _need(d_scale, "float32", "tx_dedisperse_norm d_scale")
    _need(d_offset, "float32", "tx_dedisperse_norm d_offset")
    _need(d_out, "float32", "tx_dedisperse_norm d_out")
    in_pitch = d_in.stride(0) * d_in.element_size()
    _check(_setup_norm().tx_dedisperse_norm(plan.handle, _ptr(d_in), in_pitch, int(nt), _ptr(d_scale),
                                            _ptr(d_offset), _ptr(d_out), d_out.stride(0), _stream(stream)),
           "tx_dedisperse_norm")


def tx_boxcar_snr_f32(dmt, nt, widths, snr, width, time, stream=None):
    _need(dmt, "float32", "tx_boxcar_snr_f32 dmt")
    _need_peaks((snr, width, time), "tx_boxcar_snr_f32")
    w, wp = _widths(widths)
    _check(_setup_norm().tx_boxcar_snr_f32(_ptr(dmt), dmt.shape[0], int(nt), dmt.stride(0), wp, len(w), _ptr(snr),
                                           _ptr(width), _ptr(time), _stream(stream)), "tx_boxcar_snr_f32")


def tx_boxcar_snr_fixed(dmt, nt, widths, mean, sigma, snr, width, time, stream=None):
    """Peak S/N of float32 rows with a given noise mean and sigma."""
    _need(dmt, "float32", "tx_boxcar_snr_fixed dmt")
    _need_peaks((snr, width, time), "tx_boxcar_snr_fixed")
    w, wp = _widths(widths)
    _check(_setup_norm().tx_boxcar_snr_fixed(_ptr(dmt), dmt.shape[0], int(nt), dmt.stride(0), wp, len(w),
                                             float(mean), float(sigma), _ptr(snr), _ptr(width), _ptr(time),
                                             _stream(stream)), "tx_boxcar_snr_fixed")


def tx_candidates_f32(dmt, nt, widths, gamma, cands, count, peaks=None, stream=None):
    """As tx_candidates, for a float32 DM x time tensor."""
    _need(dmt, "float32", "tx_candidates_f32 dmt")
    _need(count, "int64", "tx_candidates_f32 count")
    _need_peaks(peaks, "tx_candidates_f32")
    w, wp = _widths(widths)
    cap = (cands.numel() * cands.element_size()) // CAND_DTYPE.itemsize
    p = (ctypes.c_void_p(0),) * 3 if peaks is None else tuple(_ptr(t) for t in peaks)
    _check(_setup_norm().tx_candidates_f32(_ptr(dmt), dmt.shape[0], int(nt), dmt.stride(0), wp, len(w),
                                           float(gamma), _ptr(cands), cap, _ptr(count), *p,
                                           _stream(stream)), "tx_candidates_f32")


TX_NOALLOC_SCRATCH_BYTES = 256 << 20


def tx_dedisperse_noalloc(plan, d_in, nt, d_out, stream=None):
    """tx_dedisperse through the library's fixed scratch (no allocation)."""
    _need(d_in, "uint8", "tx_dedisperse_noalloc d_in")
    _need(d_out, "int32", "tx_dedisperse_noalloc d_out")
    in_pitch = d_in.stride(0) * d_in.element_size()
    _check(lib().tx_dedisperse_noalloc(plan.handle, _ptr(d_in), in_pitch, int(nt), _ptr(d_out), d_out.stride(0),
                                       _stream(stream)), "tx_dedisperse_noalloc")


def tx_transpose_tf(d_tf, nchan, nt, d_ft, stream=None):
    """d_tf: uint8 device tensor [>= nt, >= nchan] (time-major); d_ft: uint8
    device tensor [>= nchan, >= nt] receiving d_ft[c, t] = d_tf[t, c]."""
    _need(d_tf, "uint8", "tx_transpose_tf d_tf")
    _need(d_ft, "uint8", "tx_transpose_tf d_ft")
    _check(lib().tx_transpose_tf(_ptr(d_tf), d_tf.stride(0) * d_tf.element_size(), int(nchan), int(nt), _ptr(d_ft),
                                 d_ft.stride(0) * d_ft.element_size(), _stream(stream)), "tx_transpose_tf")


def tx_channel_power_sums(d_in, nchan, nt, d_sums, stream=None):
    """d_in: uint8 device tensor [nchan, >= nt]; d_sums: int64 device tensor
    [nchan, 4] receiving sum x, x^2, x^3, x^4 per channel (as uint64 bits)."""
    _need(d_in, "uint8", "tx_channel_power_sums d_in")
    _need(d_sums, "int64", "tx_channel_power_sums d_sums")
    _check(lib().tx_channel_power_sums(_ptr(d_in), d_in.stride(0) * d_in.element_size(), int(nchan), int(nt),
                                       _ptr(d_sums), _stream(stream)), "tx_channel_power_sums")


def tx_skf_mask(sums, nt, threshold):
    """Host: channel mask (uint8, 1 keep / 0 drop) from power sums [nchan, 4]."""
    s = np.ascontiguousarray(sums).view(np.uint64).reshape(-1, 4)
    m = np.empty(s.shape[0], dtype=np.uint8)
    _check(lib().tx_skf_mask(s.ctypes.data_as(ctypes.c_void_p), s.shape[0], int(nt), float(threshold),
                             m.ctypes.data_as(ctypes.c_void_p)), "tx_skf_mask")
    return m


def tx_cluster(plan, cands, n, radius, min_pts, stream=None):
    """DBSCAN of the first n candidate records of the device tensor ``cands``
    (int64 [>= n, 3], as filled by tx_candidates).  Returns device tensors
    (sorted records [n, 3], labels int32 [n], reps int64 [n], nclusters
    int64 [1])."""
    _need(cands, "int64", "tx_cluster cands")
    import torch
    n = int(n)
    dev = cands.device
    srt = torch.empty((max(n, 1), 3), dtype=torch.int64, device=dev)
    lab = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    rep = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    ncl = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(lib().tx_cluster(plan.handle, _ptr(cands), n, float(radius), int(min_pts), _ptr(srt), _ptr(lab), _ptr(rep),
                            _ptr(ncl), _stream(stream)), "tx_cluster")
    return srt[:n], lab[:n], rep[:n], ncl


def tx_downsample(d_in, nchan, nt_out, k, d_out, stream=None):
    """d_in: uint8 device tensor [nchan, >= k*nt_out]; d_out: uint8 device
    tensor [nchan, >= nt_out] receiving the rounded means of k samples."""
    _need(d_in, "uint8", "tx_downsample d_in")
    _need(d_out, "uint8", "tx_downsample d_out")
    _check(lib().tx_downsample(_ptr(d_in), d_in.stride(0) * d_in.element_size(), int(nchan), int(nt_out), int(k),
                               _ptr(d_out), d_out.stride(0) * d_out.element_size(), _stream(stream)), "tx_downsample")


class Ranges:
    """A dedispersion plan in DM ranges: plans[r] runs on the block
    downsampled by factors[r] (tx_ranges_*)."""

    def __init__(self, plans, factors):
        self.plans = list(plans)
        self.factors = [int(k) for k in factors]
        hs = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        ks = (ctypes.c_int32 * len(self.factors))(*self.factors)
        h = ctypes.c_void_p()
        _check(lib().tx_ranges_create(hs, ks, len(self.plans), ctypes.byref(h)), "tx_ranges_create")
        self._h = h

    def input_len(self, nt):
        n = ctypes.c_int64()
        _check(lib().tx_ranges_input_len(self._h, int(nt), ctypes.byref(n)), "tx_ranges_input_len")
        return n.value

    def dedisperse(self, d_in, nt, d_outs, stream=None):
        """d_in: uint8 device tensor [nchan, >= input_len(nt)]; d_outs[r]: int32
        device tensor [plans[r].ndm, >= nt / factors[r]]."""
        _need(d_in, "uint8", "Ranges.dedisperse d_in")
        for o in d_outs:
            _need(o, "int32", "Ranges.dedisperse d_outs")
        outs = (ctypes.c_void_p * len(d_outs))(*[_ptr(o) for o in d_outs])
        pitches = (ctypes.c_int64 * len(d_outs))(*[o.stride(0) for o in d_outs])
        _check(lib().tx_ranges_dedisperse(self._h, _ptr(d_in), d_in.stride(0) * d_in.element_size(), int(nt), outs,
                                          pitches, _stream(stream)), "tx_ranges_dedisperse")

    def close(self):
        if self._h is not None and self._h.value:
            lib().tx_ranges_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _widths(widths):
    w = np.ascontiguousarray(widths, dtype=np.int32)
    return w, w.ctypes.data_as(_c_i32p)


def tx_boxcar_snr(dmt, nt, widths, snr, width, time, stream=None):
    """dmt: int32 device tensor [ndm, pitch]; outputs float64/int32/int64 device [ndm]."""
    _need(dmt, "int32", "tx_boxcar_snr dmt")
    _need_peaks((snr, width, time), "tx_boxcar_snr")
    w, wp = _widths(widths)
    _check(lib().tx_boxcar_snr(_ptr(dmt), dmt.shape[0], int(nt), dmt.stride(0), wp, len(w), _ptr(snr),
                               _ptr(width), _ptr(time), _stream(stream)), "tx_boxcar_snr")


def tx_candidates(dmt, nt, widths, gamma, cands, count, peaks=None, stream=None):
    """cands: device tensor of at least cap*24 bytes (uint8 [cap, 24] or int64 [cap, 3]);
    count: int64 device tensor [1]; peaks: optional (snr, width, time) device tensors."""
    _need(dmt, "int32", "tx_candidates dmt")
    _need(count, "int64", "tx_candidates count")
    _need_peaks(peaks, "tx_candidates")
    w, wp = _widths(widths)
    cap = (cands.numel() * cands.element_size()) // CAND_DTYPE.itemsize
    if peaks is None:
        p = (ctypes.c_void_p(0),) * 3
    else:
        p = tuple(_ptr(t) for t in peaks)
    _check(lib().tx_candidates(_ptr(dmt), dmt.shape[0], int(nt), dmt.stride(0), wp, len(w), float(gamma),
                               _ptr(cands), cap, _ptr(count), *p, _stream(stream)), "tx_candidates")


def parse_candidates(raw, count):
    """Host view of candidate records (first min(count, cap) of them), sorted by (dm_index, time)."""
    buf = np.ascontiguousarray(raw).view(np.uint8).reshape(-1)
    rec = buf[: (buf.size // CAND_DTYPE.itemsize) * CAND_DTYPE.itemsize].view(CAND_DTYPE)
    rec = rec[: min(int(count), rec.size)].copy()
    return np.sort(rec, order=["dm_index", "time"])


def tx_profile_enable(on=True):
    _check(lib().tx_profile_enable(1 if on else 0), "tx_profile_enable")


def tx_profile_collect(kernel):
    """(total milliseconds, launches) of one kernel since the last collect."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().tx_profile_collect(int(kernel), ctypes.byref(ms), ctypes.byref(n)), "tx_profile_collect")
    return ms.value, n.value


def tx_tile_variants(stage):
    """[(outputs per tile, trials per wave)] of each variant of a stage (1 or 2)."""
    n = ctypes.c_int32()
    _check(lib().tx_tile_variants(int(stage), ctypes.byref(n)), "tx_tile_variants")
    out = []
    for v in range(n.value):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().tx_tile_variant_info(int(stage), v, ctypes.byref(a), ctypes.byref(b)), "tx_tile_variant_info")
        out.append((a.value, b.value))
    return out


# ---------------------------------------------------------------------------
# Streams and batches
# ---------------------------------------------------------------------------

class BatchBoxcar(ctypes.Structure):
    _fields_ = [("widths", ctypes.POINTER(ctypes.c_int32)), ("nw", ctypes.c_int32), ("gamma", ctypes.c_double),
                ("d_snr", ctypes.c_void_p), ("d_width", ctypes.c_void_p), ("d_time", ctypes.c_void_p),
                ("d_cands", ctypes.c_void_p), ("cap", ctypes.c_int64), ("d_count", ctypes.c_void_p)]


TX_BATCH_GRAPH = 1

_SIGS2 = {
    "tx_stream_open": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p)]),
    "tx_stream_push": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "tx_stream_push_tf": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "tx_transpose_tf": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "tx_plan_set_mask": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tx_plan_get_mask": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tx_channel_power_sums": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "tx_skf_mask": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_void_p]),
    "tx_cluster": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "tx_downsample": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "tx_ranges_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "tx_ranges_input_len": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "tx_ranges_dedisperse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                            ctypes.c_void_p]),
    "tx_ranges_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "tx_stream_position": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int64)]),
    "tx_stream_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "tx_stream_snapshot": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_void_p]),
    "tx_stream_restore": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_void_p]),
    "tx_stream_close": (ctypes.c_int, [ctypes.c_void_p]),
    "tx_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]),
    "tx_batch_clear": (ctypes.c_int, [ctypes.c_void_p]),
    "tx_batch_add": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.POINTER(BatchBoxcar)]),
    "tx_batch_add_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.POINTER(BatchBoxcar)]),
    "tx_batch_add_stream_tf": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.POINTER(BatchBoxcar)]),
    "tx_batch_stream_output": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "tx_batch_reserve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                        ctypes.c_int32]),
    "tx_plan_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "tx_pool_trim": (ctypes.c_int, []),
    "tx_batch_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tx_batch_wait": (ctypes.c_int, [ctypes.c_void_p]),
    "tx_batch_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "tx_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}
_SIGS.update(_SIGS2)


def _setup_more():
    L = lib()
    for name, (res, args) in _SIGS2.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def tx_pool_trim():
    """Give pooled scratch of the current device back to the system."""
    _check(_setup_more().tx_pool_trim(), "tx_pool_trim")


class Stream:
    """Owner of a tx_stream_t: a beam's device-resident overlap history."""

    def __init__(self, plan, max_block):
        self.plan = plan
        self.max_block = int(max_block)
        h = ctypes.c_void_p()
        _check(_setup_more().tx_stream_open(plan.handle, self.max_block, ctypes.byref(h)), "tx_stream_open")
        self._h = h

    @property
    def handle(self):
        return self._h

    def push(self, block, nt, d_out, stream=None):
        """block: uint8 tensor [nchan, >= nt] on the device or in (pinned) host memory."""
        _need(block, "uint8", "Stream.push block")
        _need(d_out, "int32", "Stream.push d_out")
        on_dev = 1 if block.is_cuda else 0
        n = ctypes.c_int64()
        _check(lib().tx_stream_push(self._h, _ptr(block), block.stride(0) * block.element_size(), int(nt), on_dev,
                                    _ptr(d_out), d_out.stride(0), ctypes.byref(n), _stream(stream)),
               "tx_stream_push")
        return n.value

    def push_tf(self, block, nt, d_out, stream=None):
        """block: time-major uint8 tensor [>= nt, >= nchan] (one row of channels
        per time sample) on the device or in (pinned) host memory."""
        _need(block, "uint8", "Stream.push_tf block")
        _need(d_out, "int32", "Stream.push_tf d_out")
        on_dev = 1 if block.is_cuda else 0
        n = ctypes.c_int64()
        _check(lib().tx_stream_push_tf(self._h, _ptr(block), block.stride(0) * block.element_size(), int(nt), on_dev,
                                       _ptr(d_out), d_out.stride(0), ctypes.byref(n), _stream(stream)),
               "tx_stream_push_tf")
        return n.value

    def position(self):
        r, e = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tx_stream_position(self._h, ctypes.byref(r), ctypes.byref(e)), "tx_stream_position")
        return r.value, e.value

    def reset(self):
        _check(lib().tx_stream_reset(self._h), "tx_stream_reset")

    def snapshot(self, stream=None):
        nchan = self.plan.nchan
        buf = np.zeros(nchan * max(self.plan.overlap, 1), dtype=np.uint8)
        held, rec, emi = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tx_stream_snapshot(self._h, buf.ctypes.data_as(ctypes.c_void_p), ctypes.byref(held),
                                        ctypes.byref(rec), ctypes.byref(emi), _stream(stream)), "tx_stream_snapshot")
        return buf[: nchan * held.value].reshape(nchan, held.value).copy(), held.value, rec.value, emi.value

    def restore(self, hist, held, received, emitted, stream=None):
        h = np.ascontiguousarray(hist, dtype=np.uint8)
        _check(lib().tx_stream_restore(self._h, h.ctypes.data_as(ctypes.c_void_p), int(held), int(received),
                                       int(emitted), _stream(stream)), "tx_stream_restore")

    def close(self):
        if self._h is not None and self._h.value:
            lib().tx_stream_close(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _box(widths, gamma, peaks, cands, count):
    _need_peaks(peaks, "batch boxcar")
    _need(count, "int64", "batch boxcar count")
    if peaks is None:
        return None, None
    w = np.ascontiguousarray(widths, dtype=np.int32)
    cap = 0 if cands is None else (cands.numel() * cands.element_size()) // CAND_DTYPE.itemsize
    bx = BatchBoxcar(w.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(w), float(gamma),
                     peaks[0].data_ptr(), peaks[1].data_ptr(), peaks[2].data_ptr(),
                     0 if cands is None else cands.data_ptr(), cap, 0 if count is None else count.data_ptr())
    return bx, w


class Batch:
    """Owner of a tx_batch_t."""

    def __init__(self, max_jobs, graph=False):
        h = ctypes.c_void_p()
        _check(_setup_more().tx_batch_create(int(max_jobs), TX_BATCH_GRAPH if graph else 0, ctypes.byref(h)),
               "tx_batch_create")
        self._h = h
        self._keep = []

    def clear(self):
        _check(lib().tx_batch_clear(self._h), "tx_batch_clear")
        self._keep = []

    def add(self, plan, d_in, nt, d_out, widths=None, gamma=6.0, peaks=None, cands=None, count=None):
        _need(d_in, "uint8", "Batch.add d_in")
        _need(d_out, "int32", "Batch.add d_out")
        bx, w = _box(widths, gamma, peaks, cands, count)
        self._keep.append(w)
        _check(lib().tx_batch_add(self._h, plan.handle, _ptr(d_in), d_in.stride(0) * d_in.element_size(), int(nt),
                                  _ptr(d_out), d_out.stride(0), None if bx is None else ctypes.byref(bx)),
               "tx_batch_add")

    def add_stream(self, stream_obj, block, nt, d_out, widths=None, gamma=6.0, peaks=None, cands=None, count=None):
        _need(block, "uint8", "Batch.add_stream block")
        _need(d_out, "int32", "Batch.add_stream d_out")
        bx, w = _box(widths, gamma, peaks, cands, count)
        self._keep.append(w)
        _check(lib().tx_batch_add_stream(self._h, stream_obj.handle, _ptr(block),
                                         block.stride(0) * block.element_size(), int(nt),
                                         1 if block.is_cuda else 0, _ptr(d_out), d_out.stride(0),
                                         None if bx is None else ctypes.byref(bx)), "tx_batch_add_stream")

    def add_stream_tf(self, stream_obj, block, nt, d_out, widths=None, gamma=6.0, peaks=None, cands=None,
                      count=None):
        """add_stream for a time-major block [>= nt, >= nchan]."""
        _need(block, "uint8", "Batch.add_stream_tf block")
        _need(d_out, "int32", "Batch.add_stream_tf d_out")
        bx, w = _box(widths, gamma, peaks, cands, count)
        self._keep.append(w)
        _check(lib().tx_batch_add_stream_tf(self._h, stream_obj.handle, _ptr(block),
                                            block.stride(0) * block.element_size(), int(nt),
                                            1 if block.is_cuda else 0, _ptr(d_out), d_out.stride(0),
                                            None if bx is None else ctypes.byref(bx)), "tx_batch_add_stream_tf")

    def reserve(self, plan, nw, max_nt, count=1):
        """Size a graph captured later for ``count`` jobs of ``plan`` with up to
        ``max_nt`` outputs and ``nw`` boxcar widths per launch."""
        _check(lib().tx_batch_reserve(self._h, plan.handle, int(nw), int(max_nt), int(count)), "tx_batch_reserve")

    def stream_output(self, job):
        n = ctypes.c_int64()
        _check(lib().tx_batch_stream_output(self._h, int(job), ctypes.byref(n)), "tx_batch_stream_output")
        return n.value

    def launch(self, stream=None):
        _check(lib().tx_batch_launch(self._h, _stream(stream)), "tx_batch_launch")

    def wait(self):
        """Block until the last launch has finished (raises on a device error)."""
        _check(lib().tx_batch_wait(self._h), "tx_batch_wait")

    def done(self):
        """True once the last launch has finished (no blocking)."""
        d = ctypes.c_int32()
        _check(lib().tx_batch_query(self._h, ctypes.byref(d)), "tx_batch_query")
        return bool(d.value)

    def close(self):
        if self._h is not None and self._h.value:
            lib().tx_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
