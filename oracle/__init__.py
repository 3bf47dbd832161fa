"""Test-only oracle for the RFIm sigma cuts (arXiv:2001.03389, Section IV)
and for the dedispersion search stage that follows them (Eq. 2).

Plain single-threaded C implementations (``rfim_oracle.c``, exact;
``dedisp_oracle.c``) behind a ctypes wrapper.  This package is test infrastructure: only the tests, the
smoke check and the benchmark's CPU-baseline leg may import it.  It shares no
code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build

_DT = {np.dtype(np.uint8): 0, np.dtype(np.float32): 1}
_lib = None


class _Step(ctypes.Structure):
    _fields_ = [("domain", ctypes.c_int32), ("replace", ctypes.c_int32),
                ("k", ctypes.c_double), ("bin_size", ctypes.c_int64)]


def _bind(path):
    lib = ctypes.CDLL(path)
    i64, vp, dbl, i32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    lib.oracle_pipeline.argtypes = [i32, vp, vp, i64, i64, i64, ctypes.POINTER(_Step), i32, vp]
    lib.oracle_pipeline.restype = i32
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        i64, vp, dbl, i32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_int
        lib.oracle_pipeline.argtypes = [i32, vp, vp, i64, i64, i64, ctypes.POINTER(_Step), i32, vp]
        lib.oracle_pipeline.restype = i32
        lib.oracle_td_step.argtypes = [i32, vp, i64, i64, i64, dbl, i32, vp, i32]
        lib.oracle_td_step.restype = i32
        lib.oracle_fd_step.argtypes = [i32, vp, i64, i64, i64, dbl, i64, i32, vp, i32]
        lib.oracle_fd_step.restype = i32
        lib.oracle_mean_f32.argtypes = [vp, i64]
        lib.oracle_mean_f32.restype = ctypes.c_float
        lib.oracle_mean_u8.argtypes = [vp, i64]
        lib.oracle_mean_u8.restype = ctypes.c_uint8
        lib.oracle_dedisp_delays.argtypes = [i64, dbl, dbl, dbl, vp, ctypes.c_int32, vp]
        lib.oracle_dedisp_delays.restype = i32
        lib.oracle_dedisperse.argtypes = [i32, vp, i64, i64, i64, vp, ctypes.c_int32, i64, vp]
        lib.oracle_dedisperse.restype = i32
        lib.oracle_series_stats.argtypes = [i32, vp, ctypes.c_int32, i64, vp, vp, vp, vp, vp]
        lib.oracle_series_stats.restype = i32
        _lib = lib
    return _lib


def _step_tuple(s):
    """Accept synth.Step-like objects or (domain, k, replace, bin) tuples."""
    if hasattr(s, "domain"):
        return s.domain, s.k, s.replace, s.bin_size
    return tuple(s)


def make_steps(steps):
    arr = (_Step * max(1, len(steps)))()
    for i, s in enumerate(steps):
        dom, k, rep, b = _step_tuple(s)
        arr[i].domain = {"td": 0, "fd": 1, "td_masked": 2}[dom]
        arr[i].replace = {"mean": 0, "median": 1}[rep]
        arr[i].k = float(k)
        arr[i].bin_size = int(b) if dom == "fd" else 0
    return arr


def pipeline(x: np.ndarray, steps, want_flags: bool = False, nsamp: int | None = None, _lib_override=None):
    """Run the step list on one beam ``x`` of shape [C][stride] (uint8 or
    float32).  Returns (out, flags or None).  ``nsamp`` < stride leaves the
    padding columns untouched."""
    x = np.ascontiguousarray(x)
    if x.dtype not in _DT:
        raise TypeError("oracle supports uint8 and float32")
    C, stride = x.shape
    T = stride if nsamp is None else int(nsamp)
    out = x.copy()
    flags = np.zeros((C, stride), dtype=np.uint8) if want_flags else None
    st = make_steps(steps)
    lib = _lib_override if _lib_override is not None else _load()
    rc = lib.oracle_pipeline(_DT[x.dtype], out.ctypes.data, out.ctypes.data, C, T, stride, st,
                                 len(steps), flags.ctypes.data if want_flags else None)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out, flags


def td_step(x, k, replace="mean"):
    return pipeline(x, [("td", k, replace, 0)], want_flags=True)


def fd_step(x, k, bin_size=32, replace="mean"):
    return pipeline(x, [("fd", k, replace, bin_size)], want_flags=True)


def mean_f32(x: np.ndarray) -> np.float32:
    x = np.ascontiguousarray(x, dtype=np.float32)
    return np.float32(_load().oracle_mean_f32(x.ctypes.data, x.size))


def mean_u8(x: np.ndarray) -> int:
    x = np.ascontiguousarray(x, dtype=np.uint8)
    return int(_load().oracle_mean_u8(x.ctypes.data, x.size))


def dedisp_delays(nchan: int, f_low_mhz: float, chan_bw_mhz: float, tsamp_s: float, dms) -> np.ndarray:
    """Eq. 2 delays in samples, int32 [ndm][nchan] (channel 0 lowest, reference
    = top channel centre, nearest sample, ties to even)."""
    dms = np.ascontiguousarray(dms, dtype=np.float64)
    out = np.zeros((dms.size, nchan), dtype=np.int32)
    rc = _load().oracle_dedisp_delays(nchan, f_low_mhz, chan_bw_mhz, tsamp_s, dms.ctypes.data, dms.size,
                                      out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the dedispersion arguments")
    return out


def dedisperse(x: np.ndarray, delays: np.ndarray, nsamp: int | None = None) -> np.ndarray:
    """Dedispersed series [ndm][nout] of beam x [C][stride]: int64 sums for
    uint8 input, double sums in channel order for float32 input."""
    x = np.ascontiguousarray(x)
    delays = np.ascontiguousarray(delays, dtype=np.int32)
    C, stride = x.shape
    T = stride if nsamp is None else int(nsamp)
    nout = T - int(delays.max())
    out = np.zeros((delays.shape[0], max(nout, 1)), dtype=np.int64 if x.dtype == np.uint8 else np.float64)
    rc = _load().oracle_dedisperse(_DT[x.dtype], x.ctypes.data, C, T, stride, delays.ctypes.data,
                                   delays.shape[0], nout, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the dedispersion arguments")
    return out


def series_stats(series: np.ndarray) -> dict:
    """Per series (row): snr, peak, peak_t, mean, std."""
    series = np.ascontiguousarray(series)
    nd, n = series.shape
    dt = 0 if series.dtype == np.int64 else 1
    if dt == 1:
        series = series.astype(np.float64)
    r = {k: np.zeros(nd, dtype=np.float64) for k in ("snr", "peak", "mean", "std")}
    r["peak_t"] = np.zeros(nd, dtype=np.int64)
    rc = _load().oracle_series_stats(dt, series.ctypes.data, nd, n, r["snr"].ctypes.data, r["peak"].ctypes.data,
                                     r["peak_t"].ctypes.data, r["mean"].ctypes.data, r["std"].ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the series")
    return r
