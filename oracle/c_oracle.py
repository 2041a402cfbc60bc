"""ctypes front end of the C oracle (``oracle/c/tx_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  A second, independent
implementation of the definitions in ``ref.py``, with OpenMP threads; the tests
pin it to the NumPy oracle and to brute force, and the benchmark times it as
the CPU baseline."""

import ctypes

import numpy as np

from .c import build as _build

_lib = None
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        L = ctypes.CDLL(path)
        L.txo_group_rule.restype = ctypes.c_int
        L.txo_group_rule.argtypes = [_f64p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.txo_plan_tables.restype = ctypes.c_int
        L.txo_plan_tables.argtypes = [_f64p, ctypes.c_int, ctypes.c_double, _f64p, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, _i64p, _i64p, _i64p, _i64p]
        L.txo_dedisperse_brute.restype = ctypes.c_int
        L.txo_dedisperse_brute.argtypes = [_f64p, ctypes.c_int, ctypes.c_double, _f64p, ctypes.c_int, _u8p,
                                           ctypes.c_int64, ctypes.c_int64, _i32p, ctypes.c_int64, ctypes.c_int]
        L.txo_dedisperse_subband.restype = ctypes.c_int
        L.txo_dedisperse_subband.argtypes = [_f64p, ctypes.c_int, ctypes.c_double, _f64p, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, _u8p, ctypes.c_int64, ctypes.c_int64,
                                             _i32p, ctypes.c_int64, ctypes.c_int]
        L.txo_boxcar_peaks.restype = ctypes.c_int
        L.txo_boxcar_peaks.argtypes = [_i32p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _i32p, ctypes.c_int,
                                       _f64p, _i32p, _i64p, ctypes.c_int]
        L.txo_candidates.restype = ctypes.c_int64
        L.txo_candidates.argtypes = [_i32p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _i32p, ctypes.c_int,
                                     ctypes.c_double, _i32p, _i64p, _i32p, _f64p, ctypes.c_int64, ctypes.c_int]
        L.txo_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def max_threads():
    return lib().txo_max_threads()


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def group_size_rule(freqs, nsub, ndm):
    f = _f64(freqs)
    return lib().txo_group_rule(_p(f, _f64p), f.shape[0], int(nsub), int(ndm))


def plan_tables(freqs, tsamp, dms, nsub, g):
    """(D(c_j, f_ch) [ngroups, nchan], D(c_j, f_s) [ngroups, nsub], D(dm_i, f_s) [ndm, nsub], overlap)."""
    f, d = _f64(freqs), _f64(dms)
    nchan, ndm = f.shape[0], d.shape[0]
    ng = (ndm + g - 1) // g
    cc = np.zeros((ng, nchan), np.int64)
    cs = np.zeros((ng, nsub), np.int64)
    fs = np.zeros((ndm, nsub), np.int64)
    o = ctypes.c_int64()
    rc = lib().txo_plan_tables(_p(f, _f64p), nchan, float(tsamp), _p(d, _f64p), ndm, int(nsub), int(g),
                               _p(cc, _i64p), _p(cs, _i64p), _p(fs, _i64p), ctypes.byref(o))
    if rc:
        raise ValueError(f"txo_plan_tables: {rc}")
    return cc, cs, fs, o.value


def _threads(threads):
    return int(threads) if threads else max_threads()


def dedisperse_subband(x, freqs, tsamp, dms, nsub, g, nt, threads=None):
    f, d = _f64(freqs), _f64(dms)
    x = np.ascontiguousarray(x, dtype=np.uint8)
    y = np.zeros((d.shape[0], int(nt)), np.int32)
    rc = lib().txo_dedisperse_subband(_p(f, _f64p), f.shape[0], float(tsamp), _p(d, _f64p), d.shape[0], int(nsub),
                                      int(g), _p(x, _u8p), x.shape[1], int(nt), _p(y, _i32p), int(nt),
                                      _threads(threads))
    if rc:
        raise ValueError(f"txo_dedisperse_subband: {rc}")
    return y


def dedisperse_brute(x, freqs, tsamp, dms, nt, threads=None):
    f, d = _f64(freqs), _f64(dms)
    x = np.ascontiguousarray(x, dtype=np.uint8)
    y = np.zeros((d.shape[0], int(nt)), np.int32)
    lib().txo_dedisperse_brute(_p(f, _f64p), f.shape[0], float(tsamp), _p(d, _f64p), d.shape[0], _p(x, _u8p),
                               x.shape[1], int(nt), _p(y, _i32p), int(nt), _threads(threads))
    return y


def boxcar_peaks(Y, widths, threads=None):
    Y = np.ascontiguousarray(Y, dtype=np.int32)
    w = np.ascontiguousarray(sorted(int(v) for v in widths), dtype=np.int32)
    n = Y.shape[0]
    snr, wid, tim = np.zeros(n), np.zeros(n, np.int32), np.zeros(n, np.int64)
    lib().txo_boxcar_peaks(_p(Y, _i32p), n, Y.shape[1], Y.shape[1], _p(w, _i32p), len(w), _p(snr, _f64p),
                           _p(wid, _i32p), _p(tim, _i64p), _threads(threads))
    return snr, wid, tim


def boxcar_candidates(Y, widths, gamma, threads=None, cap=1 << 22):
    """List of (d, t, width, snr) in (d, t) order, as ``ref.boxcar_candidates``."""
    Y = np.ascontiguousarray(Y, dtype=np.int32)
    w = np.ascontiguousarray(sorted(int(v) for v in widths), dtype=np.int32)
    cd, ct = np.zeros(cap, np.int32), np.zeros(cap, np.int64)
    cw, cs = np.zeros(cap, np.int32), np.zeros(cap)
    n = lib().txo_candidates(_p(Y, _i32p), Y.shape[0], Y.shape[1], Y.shape[1], _p(w, _i32p), len(w), float(gamma),
                             _p(cd, _i32p), _p(ct, _i64p), _p(cw, _i32p), _p(cs, _f64p), cap, _threads(threads))
    if n > cap:
        raise ValueError("candidate capacity exceeded")
    return [(int(cd[k]), int(ct[k]), int(cw[k]), float(cs[k])) for k in range(n)]
