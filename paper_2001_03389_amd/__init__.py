"""Python binding of librfim (include/rfim.h): RFI mitigation by iterated
time- and frequency-domain sigma cuts (RFIm, arXiv:2001.03389, Section IV) on
MI355X.

Argument marshalling only: every step runs in the HIP kernels of librfim.so.
Tensors are torch CUDA (HIP) tensors of shape [nchan][row_stride] (uint8 or
float32, unit stride along time); ``nsamp`` <= row_stride samples per row are
processed.  Calls are asynchronous on the given (or current) stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librfim.so")

RFIM_OK, RFIM_ERR_INVALID_ARG, RFIM_ERR_UNSUPPORTED = 0, -1, -2
RFIM_ERR_OUT_OF_MEMORY, RFIM_ERR_DEVICE, RFIM_ERR_BUDGET, RFIM_ERR_MISMATCH = -3, -4, -5, -6
RFIM_ERR_SCRATCH = -7
RFIM_NOALLOC_SCRATCH_BYTES = 32 << 20
RFIM_U8, RFIM_F32 = 0, 1
RFIM_REPLACE_MEAN, RFIM_REPLACE_MEDIAN = 0, 1
RFIM_TD, RFIM_FD, RFIM_TD_MASKED = 0, 1, 2
RFIM_KERNEL_TD_ROWS_U8, RFIM_KERNEL_FUSED_U8 = 0, 1
RFIM_KERNEL_TD_ROWS_F32, RFIM_KERNEL_FUSED_F32, RFIM_KERNEL_TD_WIDE_F32, RFIM_KERNEL_FD_WIDE_F32 = 2, 3, 4, 5
RFIM_KERNEL_TD_TWO_F32, RFIM_KERNEL_FD_TWO_F32 = 6, 7
RFIM_KERNEL_PERSIST_U8 = 8
KERNEL_NAMES = {RFIM_KERNEL_TD_ROWS_U8: "k_td_rows_u8", RFIM_KERNEL_FUSED_U8: "k_fused_u8",
                RFIM_KERNEL_TD_ROWS_F32: "k_td_rows_f32", RFIM_KERNEL_FUSED_F32: "k_fused_f32",
                RFIM_KERNEL_TD_WIDE_F32: "k_td_wide_f32", RFIM_KERNEL_FD_WIDE_F32: "k_fd_wide_f32",
                RFIM_KERNEL_TD_TWO_F32: "k_td_two_f32", RFIM_KERNEL_FD_TWO_F32: "k_fd_two_f32",
                RFIM_KERNEL_PERSIST_U8: "k_persist_u8"}


FD_PATH_NAMES = {0: "none", 1: "u8_bin32_g4", 2: "u8_bin32_g8", 3: "u8_bin32_g16", 4: "u8_vec", 5: "u8_bytes",
                 6: "f32_fast", 7: "f32_wide"}


class rfim_plan_beam_info(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("fd_path", ctypes.c_int32), ("tile_samples", ctypes.c_int32),
                ("tile_pitch", ctypes.c_int32), ("lds_bytes", ctypes.c_int64), ("td_threads", ctypes.c_int32),
                ("td_values_per_lane", ctypes.c_int32), ("fd_bin", ctypes.c_int32),
                ("fd_bins_per_lane", ctypes.c_int32)]


class RfimError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})" if what else status_string(status))


class rfim_beam(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("nchan", ctypes.c_int64), ("nsamp", ctypes.c_int64),
                ("row_stride", ctypes.c_int64), ("in_", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


class rfim_step(ctypes.Structure):
    _fields_ = [("domain", ctypes.c_int32), ("replace", ctypes.c_int32),
                ("k", ctypes.c_double), ("bin_size", ctypes.c_int64)]


RFIM_SERVE_PER_CALL, RFIM_SERVE_BATCHED, RFIM_SERVE_GRAPH = 0, 1, 2


class rfim_serve_config(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("nchan", ctypes.c_int64), ("nsamp", ctypes.c_int64),
                ("ring_depth", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64), ("max_wait_s", ctypes.c_double),
                ("deadline_s", ctypes.c_double), ("mode", ctypes.c_int32), ("mock", ctypes.c_int32),
                ("mock_launch_s", ctypes.c_double), ("mock_beam_s", ctypes.c_double)]


class rfim_serve_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "admitted", "rejected_budget", "rejected_ring",
                                                "completed", "launches", "deadline_misses", "max_backlog",
                                                "slots", "in_flight")] + \
               [(n, ctypes.c_double) for n in ("p50_s", "p99_s", "max_s", "mean_batch")]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded librfim.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2001_03389_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        st, i32, i64, vp, dbl = ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
        PB, PS = ctypes.POINTER(rfim_beam), ctypes.POINTER(rfim_step)
        L.rfim_td_sigma_cut.argtypes = [PB, i32, dbl, i32, vp]
        L.rfim_fd_sigma_cut.argtypes = [PB, i32, dbl, i64, i32, vp]
        L.rfim_pipeline_run.argtypes = [PB, i32, PS, i32, vp, vp]
        L.rfim_pipeline_run_noalloc.argtypes = [PB, i32, PS, i32, vp]
        L.rfim_plan_create.argtypes = [PB, i32, PS, i32, ctypes.c_char_p, ctypes.POINTER(vp)]
        L.rfim_plan_destroy.argtypes = [vp]
        L.rfim_plan_flag_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
        L.rfim_plan_set_timing.argtypes = [vp, i32]
        L.rfim_plan_kernel_times.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.POINTER(ctypes.c_double)]
        L.rfim_plan_capture.argtypes = [vp, PB, i32, vp]
        L.rfim_plan_replay.argtypes = [vp, vp]
        L.rfim_autotune.argtypes = [PB, i32, PS, i32, ctypes.c_char_p, vp, ctypes.POINTER(dbl)]
        L.rfim_tune_lookup.argtypes = [ctypes.c_char_p, PB, i32, PS, i32, ctypes.POINTER(i64)]
        L.rfim_tune_store.argtypes = [ctypes.c_char_p, PB, i32, PS, i32, ctypes.POINTER(i64), dbl]
        L.rfim_plan_replay_on.argtypes = [vp, PB, i32, vp]
        L.rfim_serve_create.argtypes = [ctypes.POINTER(rfim_serve_config), PS, i32, ctypes.POINTER(vp)]
        L.rfim_serve_now.argtypes = [vp]
        L.rfim_serve_now.restype = dbl
        L.rfim_serve_submit.argtypes = [vp, i32, vp, i32, vp, vp, dbl]
        L.rfim_plan_describe.argtypes = [vp, i32, i32, ctypes.POINTER(rfim_plan_beam_info)]
        L.rfim_plan_describe.restype = st
        L.rfim_serve_poll.argtypes = [vp, dbl, ctypes.POINTER(ctypes.c_uint64)]
        L.rfim_serve_drain.argtypes = [vp, dbl]
        L.rfim_serve_get_stats.argtypes = [vp, ctypes.POINTER(rfim_serve_stats)]
        L.rfim_serve_destroy.argtypes = [vp]
        for f in ("rfim_plan_replay_on", "rfim_serve_create", "rfim_serve_submit", "rfim_serve_poll",
                  "rfim_serve_drain", "rfim_serve_get_stats", "rfim_serve_destroy"):
            getattr(L, f).restype = st
        for f in ("rfim_td_sigma_cut", "rfim_fd_sigma_cut", "rfim_pipeline_run", "rfim_pipeline_run_noalloc",
                  "rfim_plan_create",
                  "rfim_plan_destroy", "rfim_plan_flag_counts", "rfim_plan_set_timing",
                  "rfim_plan_kernel_times", "rfim_plan_capture", "rfim_plan_replay", "rfim_autotune",
                  "rfim_tune_lookup", "rfim_tune_store"):
            getattr(L, f).restype = st
        L.rfim_dedisp_create.argtypes = [i64, dbl, dbl, dbl, ctypes.POINTER(dbl), i32, ctypes.POINTER(vp)]
        L.rfim_dedisp_destroy.argtypes = [vp]
        L.rfim_dedisp_delays.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.rfim_dedisperse.argtypes = [vp, PB, i64, vp, vp]
        L.rfim_series_stats.argtypes = [i32, vp, i32, i64, vp, vp]
        for f in ("rfim_dedisp_create", "rfim_dedisp_destroy", "rfim_dedisp_delays", "rfim_dedisperse",
                  "rfim_series_stats"):
            getattr(L, f).restype = st
        L.rfim_status_string.argtypes = [st]
        L.rfim_status_string.restype = ctypes.c_char_p
        L.rfim_version.argtypes = []
        L.rfim_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().rfim_status_string(int(s)).decode()


def version() -> str:
    return lib().rfim_version().decode()


def _check(rc: int, what: str):
    if rc != RFIM_OK:
        raise RfimError(rc, what)


# ---------------------------------------------------------------- marshalling
def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.uint8:
        return RFIM_U8
    if t.dtype == torch.float32:
        return RFIM_F32
    raise TypeError(f"unsupported dtype {t.dtype} (uint8 or float32)")


def make_beam(inp, out=None, flags=None, nsamp: int | None = None) -> rfim_beam:
    """Describe one beam from torch tensors [nchan][row_stride] (time fastest)."""
    if inp.dim() != 2 or inp.stride(1) != 1:
        raise ValueError("beam tensors must be 2-D [nchan][row_stride] with unit time stride")
    out = inp if out is None else out
    if out.shape != inp.shape or out.stride() != inp.stride() or out.dtype != inp.dtype:
        raise ValueError("out must match in (shape, strides, dtype)")
    C = inp.shape[0]
    stride = inp.stride(0) if C > 1 else inp.shape[1]
    T = inp.shape[1] if nsamp is None else int(nsamp)
    b = rfim_beam()
    b.dtype = _dtype_code(inp)
    b.reserved = 0
    b.nchan, b.nsamp, b.row_stride = C, T, stride
    b.in_, b.out = inp.data_ptr(), out.data_ptr()
    if flags is not None:
        if flags.dtype.itemsize != 1 or flags.shape != inp.shape or flags.stride() != inp.stride():
            raise ValueError("flags must be uint8 with the beam's shape and strides")
        b.flags = flags.data_ptr()
    else:
        b.flags = None
    return b


def _step_fields(s):
    if isinstance(s, rfim_step):
        return s.domain, s.replace, s.k, s.bin_size
    if hasattr(s, "domain"):
        dom, k, rep, binsz = s.domain, s.k, s.replace, s.bin_size
    else:
        dom, k, rep, binsz = s
    d = {"td": RFIM_TD, "fd": RFIM_FD, "td_masked": RFIM_TD_MASKED}.get(dom, dom)
    r = {"mean": RFIM_REPLACE_MEAN, "median": RFIM_REPLACE_MEDIAN}.get(rep, rep)
    return int(d), int(r), float(k), int(binsz) if int(d) == RFIM_FD else 0


def make_steps(steps: Sequence) -> ctypes.Array:
    arr = (rfim_step * max(1, len(steps)))()
    for i, s in enumerate(steps):
        arr[i].domain, arr[i].replace, arr[i].k, arr[i].bin_size = _step_fields(s)
    return arr


def _beams(inputs, outputs, flags, nsamp):
    n = len(inputs)
    outputs = list(outputs) if outputs is not None else [None] * n
    flags = list(flags) if flags is not None else [None] * n
    nsamp = list(nsamp) if isinstance(nsamp, (list, tuple)) else [nsamp] * n
    arr = (rfim_beam * max(1, n))()
    for i in range(n):
        arr[i] = make_beam(inputs[i], outputs[i], flags[i], nsamp[i])
    return arr, n


def shape_beam(dtype: str, nchan: int, nsamp: int, row_stride: int | None = None,
               flags: bool = False) -> rfim_beam:
    """A beam descriptor that carries only a shape (plans, the tuner and the
    tuning cache ignore pointers); the pointers are dummies."""
    b = rfim_beam()
    b.dtype = {"u8": RFIM_U8, "f32": RFIM_F32}.get(dtype, dtype)
    b.reserved = 0
    b.nchan, b.nsamp = int(nchan), int(nsamp)
    b.row_stride = int(row_stride if row_stride is not None else nsamp)
    b.in_ = b.out = 4096
    b.flags = 8192 if flags else None
    return b


def _shape_array(shapes):
    arr = (rfim_beam * max(1, len(shapes)))()
    for i, b in enumerate(shapes):
        arr[i] = b
    return arr


RFIM_TUNE_NPARAMS = 6


def tune_lookup(path: str, shapes: Sequence[rfim_beam], steps: Sequence):
    """(uint8 tile cap, float32 LDS bytes, float32 tile cap, uint8 LDS bytes,
    uint8 schedule, uint8 TD rows per work-group) stored in the tuning cache
    for these shapes and steps, or None (rfim_tune_lookup)."""
    out = (ctypes.c_int64 * RFIM_TUNE_NPARAMS)()
    rc = lib().rfim_tune_lookup(path.encode(), _shape_array(shapes), len(shapes), make_steps(steps),
                                len(steps), out)
    if rc == RFIM_ERR_UNSUPPORTED:
        return None
    _check(rc, "rfim_tune_lookup")
    return tuple(int(v) for v in out)


def tune_store(path: str, shapes: Sequence[rfim_beam], steps: Sequence, params, ms: float = 0.0) -> None:
    """Adds or replaces the cache entry of these shapes and steps (rfim_tune_store)."""
    vals = [int(v) for v in params]
    defaults = [64, 81920, 64, 51200, 0, 4]   # the uint8 LDS budget, schedule and TD rows may be left out
    if not 3 <= len(vals) <= RFIM_TUNE_NPARAMS:
        raise ValueError(f"3 to {RFIM_TUNE_NPARAMS} tuning parameters expected")
    vals += defaults[len(vals):]
    p = (ctypes.c_int64 * RFIM_TUNE_NPARAMS)(*vals)
    _check(lib().rfim_tune_store(path.encode(), _shape_array(shapes), len(shapes), make_steps(steps),
                                 len(steps), p, float(ms)), "rfim_tune_store")


def autotune(shapes: Sequence[rfim_beam], steps: Sequence, cache_path: str, stream=None) -> float:
    """Times the candidate kernel configurations for these shapes and steps,
    stores the fastest bit-identical one in the cache; returns its time per
    run in ms (rfim_autotune)."""
    best = ctypes.c_double()
    _check(lib().rfim_autotune(_shape_array(shapes), len(shapes), make_steps(steps), len(steps),
                               cache_path.encode(), _stream_handle(stream), ctypes.byref(best)),
           "rfim_autotune")
    return float(best.value)


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ entry points
def rfim_pipeline_run(inputs: Sequence, steps: Sequence, outputs: Sequence | None = None,
                      flags: Sequence | None = None, nsamp=None, plan: "Plan | None" = None,
                      stream=None) -> None:
    """Run ``steps`` in order on every beam (rfim_pipeline_run)."""
    arr, n = _beams(inputs, outputs, flags, nsamp)
    st = make_steps(steps)
    rc = lib().rfim_pipeline_run(arr, n, st, len(steps), plan.handle if plan else None,
                                 _stream_handle(stream))
    _check(rc, "rfim_pipeline_run")


def rfim_pipeline_run_noalloc(inputs: Sequence, steps: Sequence, outputs: Sequence | None = None,
                              flags: Sequence | None = None, nsamp=None, stream=None) -> None:
    """Run ``steps`` in order on every beam without allocating anything: the
    workspace is the library's fixed per-GPU scratch array
    (rfim_pipeline_run_noalloc).  Calls that overlap on one GPU race."""
    arr, n = _beams(inputs, outputs, flags, nsamp)
    st = make_steps(steps)
    _check(lib().rfim_pipeline_run_noalloc(arr, n, st, len(steps), _stream_handle(stream)),
           "rfim_pipeline_run_noalloc")


def rfim_td_sigma_cut(inputs: Sequence, k: float, replace="mean", outputs=None, flags=None,
                      nsamp=None, stream=None) -> None:
    """One time-domain sigma cut on every beam (rfim_td_sigma_cut)."""
    arr, n = _beams(inputs, outputs, flags, nsamp)
    r = {"mean": RFIM_REPLACE_MEAN, "median": RFIM_REPLACE_MEDIAN}.get(replace, replace)
    _check(lib().rfim_td_sigma_cut(arr, n, float(k), int(r), _stream_handle(stream)),
           "rfim_td_sigma_cut")


def rfim_fd_sigma_cut(inputs: Sequence, k: float, bin_size: int = 32, replace="mean",
                      outputs=None, flags=None, nsamp=None, stream=None) -> None:
    """One frequency-domain sigma cut on every beam (rfim_fd_sigma_cut)."""
    arr, n = _beams(inputs, outputs, flags, nsamp)
    r = {"mean": RFIM_REPLACE_MEAN, "median": RFIM_REPLACE_MEDIAN}.get(replace, replace)
    _check(lib().rfim_fd_sigma_cut(arr, n, float(k), int(bin_size), int(r), _stream_handle(stream)),
           "rfim_fd_sigma_cut")


class Plan:
    """rfim_plan_create / rfim_plan_destroy / rfim_plan_flag_counts."""

    def __init__(self, inputs: Sequence, steps: Sequence, outputs=None, flags=None, nsamp=None,
                 tune_cache: str | None = None):
        arr, n = _beams(inputs, outputs, flags, nsamp)
        self.nbeams, self.nsteps = n, len(steps)
        st = make_steps(steps)
        h = ctypes.c_void_p()
        rc = lib().rfim_plan_create(arr, n, st, len(steps),
                                    tune_cache.encode() if tune_cache else None, ctypes.byref(h))
        _check(rc, "rfim_plan_create")
        self.handle = h

    def capture(self, inputs: Sequence, outputs=None, flags=None, nsamp=None, stream=None) -> None:
        """Records one run on these buffers into the plan's HIP graph (rfim_plan_capture)."""
        arr, n = _beams(inputs, outputs, flags, nsamp)
        _check(lib().rfim_plan_capture(self.handle, arr, n, _stream_handle(stream)), "rfim_plan_capture")

    def replay(self, stream=None) -> None:
        """Launches the captured graph (rfim_plan_replay)."""
        _check(lib().rfim_plan_replay(self.handle, _stream_handle(stream)), "rfim_plan_replay")

    def replay_on(self, inputs: Sequence, outputs=None, flags=None, nsamp=None, stream=None) -> None:
        """Replays the captured graph on other buffers of the same shapes (rfim_plan_replay_on)."""
        arr, n = _beams(inputs, outputs, flags, nsamp)
        _check(lib().rfim_plan_replay_on(self.handle, arr, n, _stream_handle(stream)), "rfim_plan_replay_on")

    def flag_counts(self):
        buf = (ctypes.c_uint64 * (self.nbeams * self.nsteps))()
        _check(lib().rfim_plan_flag_counts(self.handle, buf), "rfim_plan_flag_counts")
        return [[buf[b * self.nsteps + s] for s in range(self.nsteps)] for b in range(self.nbeams)]

    def describe(self, beam: int, run: int = 0) -> dict:
        """Launch configuration chosen for one beam in one run of [TD][FD]
        steps (rfim_plan_describe); ``fd_path`` is named as in FD_PATH_NAMES."""
        info = rfim_plan_beam_info()
        _check(lib().rfim_plan_describe(self.handle, int(beam), int(run), ctypes.byref(info)), "rfim_plan_describe")
        d = {n: getattr(info, n) for n, _ in rfim_plan_beam_info._fields_}
        d["fd_path"] = FD_PATH_NAMES.get(d["fd_path"], d["fd_path"])
        return d

    def set_timing(self, enable: bool = True):
        _check(lib().rfim_plan_set_timing(self.handle, 1 if enable else 0), "rfim_plan_set_timing")

    def kernel_times(self, kind: int):
        """(launches, total milliseconds) of one kernel kind since timing was enabled."""
        n = ctypes.c_uint64()
        ms = ctypes.c_double()
        _check(lib().rfim_plan_kernel_times(self.handle, int(kind), ctypes.byref(n), ctypes.byref(ms)),
               "rfim_plan_kernel_times")
        return int(n.value), float(ms.value)

    def close(self):
        if self.handle:
            lib().rfim_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Serve:
    """Streaming serve loop (rfim_serve_*): submit arrivals, poll, drain, stats.
    ``mock=True`` runs the scheduler with a modelled executor and no GPU work."""

    def __init__(self, steps: Sequence, *, dtype="u8", nchan=1536, nsamp=12500, ring_depth=2, max_batch=8,
                 hbm_budget=1 << 30, max_wait_s=0.002, deadline_s=1.024, mode="batched", mock=False,
                 mock_launch_s=0.0, mock_beam_s=0.0):
        c = rfim_serve_config()
        c.dtype = {"u8": RFIM_U8, "f32": RFIM_F32}.get(dtype, dtype)
        c.reserved = 0
        c.nchan, c.nsamp = int(nchan), int(nsamp)
        c.ring_depth, c.max_batch, c.hbm_budget = int(ring_depth), int(max_batch), int(hbm_budget)
        c.max_wait_s, c.deadline_s = float(max_wait_s), float(deadline_s)
        c.mode = {"per_call": RFIM_SERVE_PER_CALL, "batched": RFIM_SERVE_BATCHED,
                  "graph": RFIM_SERVE_GRAPH}.get(mode, mode)
        c.mock = 1 if mock else 0
        c.mock_launch_s, c.mock_beam_s = float(mock_launch_s), float(mock_beam_s)
        self.cfg = c
        h = ctypes.c_void_p()
        _check(lib().rfim_serve_create(ctypes.byref(c), make_steps(steps), len(steps), ctypes.byref(h)),
               "rfim_serve_create")
        self.handle = h

    def now(self) -> float:
        return float(lib().rfim_serve_now(self.handle))

    def _check_batch(self, t, what: str, device_only: bool = False):
        import torch
        want = torch.uint8 if self.cfg.dtype == RFIM_U8 else torch.float32
        if t.dtype != want or t.numel() != self.cfg.nchan * self.cfg.nsamp or not t.is_contiguous():
            raise ValueError(f"{what} must be a contiguous {want} tensor of {self.cfg.nchan} x {self.cfg.nsamp} "
                             f"elements (got {t.dtype}, {tuple(t.shape)}, contiguous={t.is_contiguous()})")
        if device_only and not t.is_cuda:
            raise ValueError(f"{what} must be a device tensor")

    def submit(self, beam: int, src=None, arrival_s: float = 0.0, dst=None, stream=None) -> bool:
        """True if admitted, False if refused (budget or the beam's ring full).
        ``src``: a contiguous torch tensor (device or host) holding one batch, or
        None (mock); a device src is copied after the work queued so far on
        ``stream`` (default: the current stream).  ``dst``: contiguous device
        tensor for the mitigated batch (None: in place in the pool)."""
        ptr, on_host, sstream = None, 0, None
        if src is not None:
            self._check_batch(src, "src")
            ptr, on_host = src.data_ptr(), 0 if src.is_cuda else 1
            if src.is_cuda:
                sstream = _stream_handle(stream)
        if dst is not None:
            self._check_batch(dst, "dst", device_only=True)
        rc = lib().rfim_serve_submit(self.handle, int(beam), ptr, on_host, sstream,
                                     dst.data_ptr() if dst is not None else None, float(arrival_s))
        if rc == RFIM_ERR_BUDGET:
            return False
        _check(rc, "rfim_serve_submit")
        return True

    def poll(self, now_s: float) -> int:
        n = ctypes.c_uint64()
        _check(lib().rfim_serve_poll(self.handle, float(now_s), ctypes.byref(n)), "rfim_serve_poll")
        return int(n.value)

    def drain(self, now_s: float) -> None:
        _check(lib().rfim_serve_drain(self.handle, float(now_s)), "rfim_serve_drain")

    def stats(self) -> dict:
        st = rfim_serve_stats()
        _check(lib().rfim_serve_get_stats(self.handle, ctypes.byref(st)), "rfim_serve_get_stats")
        return {n: getattr(st, n) for n, _ in rfim_serve_stats._fields_}

    def close(self):
        if self.handle:
            lib().rfim_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ dedispersion
class Dedisp:
    """Incoherent dedispersion over a list of trial DMs (rfim_dedisp_create,
    rfim_dedisperse; Eq. 2 delays relative to the top channel's centre).
    Channel c is centred at f_low + (c + 1/2) * chan_bw MHz, channel 0 lowest."""

    def __init__(self, nchan: int, dms: Sequence[float], f_low_mhz: float = 1220.0,
                 chan_bw_mhz: float | None = None, tsamp_s: float = 81.92e-6):
        import numpy as np
        bw = 300.0 / nchan if chan_bw_mhz is None else float(chan_bw_mhz)
        d = np.ascontiguousarray(dms, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().rfim_dedisp_create(int(nchan), float(f_low_mhz), bw, float(tsamp_s),
                                        d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d.size,
                                        ctypes.byref(h)), "rfim_dedisp_create")
        self.handle, self.nchan, self.ndm = h, int(nchan), int(d.size)
        mx = ctypes.c_int32()
        _check(lib().rfim_dedisp_delays(self.handle, None, ctypes.byref(mx)), "rfim_dedisp_delays")
        self.max_delay = int(mx.value)

    def delays(self):
        """Host copy of the delays, int32 [ndm][nchan] samples."""
        import numpy as np
        out = np.zeros((self.ndm, self.nchan), dtype=np.int32)
        _check(lib().rfim_dedisp_delays(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None),
               "rfim_dedisp_delays")
        return out

    def run(self, beam, nout: int | None = None, nsamp: int | None = None, series=None, stream=None):
        """Dedispersed series [ndm][nout] of a [nchan][row_stride] beam tensor:
        int32 for uint8 beams, float64 for float32 beams (rfim_dedisperse)."""
        import torch
        b = make_beam(beam, None, None, nsamp)
        n = int(b.nsamp - self.max_delay) if nout is None else int(nout)
        dt = torch.int32 if beam.dtype == torch.uint8 else torch.float64
        if series is None:
            series = torch.empty((self.ndm, max(n, 1)), dtype=dt, device=beam.device)
        elif series.dtype != dt or not series.is_contiguous() or series.numel() < self.ndm * n:
            raise ValueError(f"series must be a contiguous {dt} tensor of at least {self.ndm} x {n} values")
        _check(lib().rfim_dedisperse(self.handle, ctypes.byref(b), n, series.data_ptr(), _stream_handle(stream)),
               "rfim_dedisperse")
        return series

    def close(self):
        if self.handle:
            lib().rfim_dedisp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def series_stats(series, stream=None):
    """[nseries][5] float64 device tensor of (SNR, peak, first peak index,
    mean, std) per row of a contiguous int32 or float64 series tensor
    (rfim_series_stats)."""
    import torch
    if series.dim() != 2 or not series.is_contiguous() or series.dtype not in (torch.int32, torch.float64):
        raise ValueError("series must be a contiguous 2-D int32 or float64 tensor")
    out = torch.empty((series.shape[0], 5), dtype=torch.float64, device=series.device)
    dt = RFIM_U8 if series.dtype == torch.int32 else RFIM_F32
    _check(lib().rfim_series_stats(dt, series.data_ptr(), series.shape[0], series.shape[1], out.data_ptr(),
                                   _stream_handle(stream)), "rfim_series_stats")
    return out
