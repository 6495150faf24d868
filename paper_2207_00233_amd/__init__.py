"""MI355X implementation of Frequency Selective Extrapolation (FSE) with the
optimized, parallel block processing order of Seiler & Kaup.

This module is a thin ctypes binding of ``libfse.so`` (C ABI in
``include/fse.h``): it marshals arguments and nothing else; every step of the
extrapolation runs in the library's HIP kernels.  Importing the package does
not load the library; the first call does, and raises if the library has not
been built (``python -m paper_2207_00233_amd.build``) -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfse.so")

FSE_OK = 0
FSE_PENDING = 1
FSE_ERR_INVALID = -1
FSE_ERR_UNSUPPORTED = -2
FSE_ERR_NOMEM = -3
FSE_ERR_AGAIN = -4
FSE_ERR_DEVICE = -5
FSE_ERR_TICKET = -6

FSE_ORDER_OPTIMIZED = 0
FSE_ORDER_LINESCAN = 1
FSE_ORDER_REFINED = 2
FSE_FP64 = 0
FSE_FP32 = 1
FSE_FP32_RERANK = 2
FSE_FP32_F16X3 = 3
FSE_FLAG_DEVICE_PTRS = 1
FSE_MAX_ITERATIONS = 1024

EXPORTED = ("fse_plan", "fse_plan_destroy", "fse_conceal_image", "fse_conceal_image_noalloc",
            "fse_submit", "fse_poll", "fse_schedule", "fse_schedule_refined",
            "fse_last_call_stats", "fse_plan_get_tuning", "fse_plan_set_tuning",
            "fse_plan_serving_stats", "fse_plan3", "fse_plan3_destroy", "fse_conceal_volume",
            "fse_schedule3", "fse_measure_peaks", "fse_strerror")
FSE_NOALLOC_SCRATCH_BYTES = 128 << 20


class FseError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = "unknown"
        try:
            msg = load().fse_strerror(code).decode()
        except Exception:  # pragma: no cover
            pass
        super().__init__(f"{where}: {msg} ({code})")


class _Params(ctypes.Structure):
    _fields_ = [
        ("block_w", ctypes.c_int32), ("block_h", ctypes.c_int32),
        ("border_d", ctypes.c_int32),
        ("fft_w", ctypes.c_int32), ("fft_h", ctypes.c_int32),
        ("rho", ctypes.c_double), ("delta", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("iterations", ctypes.c_int32), ("order", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("grid_off_x", ctypes.c_int32), ("grid_off_y", ctypes.c_int32),
        ("empty_fill", ctypes.c_double),
        ("device_mem_budget", ctypes.c_int64),
        ("max_inflight_frames", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("rerank_gap", ctypes.c_double),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("lost_blocks", ctypes.c_int32),
                ("max_wave_blocks", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("latency_ms", ctypes.c_double)]


class _Trace(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int32), ("count", ctypes.c_int32),
                ("block", ctypes.POINTER(ctypes.c_int32)),
                ("wave", ctypes.POINTER(ctypes.c_int32)),
                ("u", ctypes.POINTER(ctypes.c_int32)),
                ("dc", ctypes.POINTER(ctypes.c_double))]


class _Frame(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("stride", ctypes.c_int32),
                ("lost", ctypes.c_void_p), ("lost_stride", ctypes.c_int32),
                ("out", ctypes.c_void_p), ("out_stride", ctypes.c_int32),
                ("out_f32", ctypes.c_void_p), ("out_f64", ctypes.c_void_p),
                ("trace", ctypes.POINTER(_Trace)), ("stats", ctypes.POINTER(_Stats))]


class _ServingStats(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("peak_committed", ctypes.c_int64), ("admitted_frames", ctypes.c_int64),
                ("peak_frames", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("step_blocks_cap", ctypes.c_int64), ("peak_step_blocks", ctypes.c_int64)]


class _Peaks(ctypes.Structure):
    _fields_ = [("fp32_fma_tflops", ctypes.c_double), ("fp64_fma_tflops", ctypes.c_double),
                ("lds_read_tbps", ctypes.c_double), ("hbm_copy_tbps", ctypes.c_double),
                ("compute_units", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def measure_peaks() -> dict:
    """fse_measure_peaks: the current device's measured FP32 / FP64 vector FMA
    rates (TFLOP/s), LDS read and HBM copy bandwidths (TB/s)."""
    pk = _Peaks()
    _check(load().fse_measure_peaks(ctypes.byref(pk)), "fse_measure_peaks")
    return {k: getattr(pk, k) for k, _ in _Peaks._fields_ if k != "reserved"}


class _Params3(ctypes.Structure):
    _fields_ = [("block_t", ctypes.c_int32), ("block_h", ctypes.c_int32),
                ("block_w", ctypes.c_int32), ("border_t", ctypes.c_int32),
                ("border_d", ctypes.c_int32), ("fft_t", ctypes.c_int32),
                ("fft_h", ctypes.c_int32), ("fft_w", ctypes.c_int32),
                ("rho", ctypes.c_double), ("delta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("iterations", ctypes.c_int32), ("order", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("empty_fill", ctypes.c_double)]


class _Volume(ctypes.Structure):
    _fields_ = [("volume", ctypes.c_void_p), ("lost", ctypes.c_void_p),
                ("frames", ctypes.c_int32), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("out", ctypes.c_void_p), ("out_f64", ctypes.c_void_p),
                ("stats", ctypes.POINTER(_Stats))]


class _CallStats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("launches", ctypes.c_int64),
                ("blocks", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("transform_ms", ctypes.c_double), ("span_ms", ctypes.c_double),
                ("groups", ctypes.c_int64), ("busy_ms", ctypes.c_double),
                ("rescored", ctypes.c_int64), ("rescore_candidates", ctypes.c_int64),
                ("rescore_wide", ctypes.c_int64), ("rescore_max_wave", ctypes.c_int64)]


class _Tuning(ctypes.Structure):
    _fields_ = [("wave_threshold_16", ctypes.c_int32), ("wave_threshold_8", ctypes.c_int32),
                ("frame_groups", ctypes.c_int32), ("crit_depth", ctypes.c_double),
                ("crit_prio", ctypes.c_int32), ("crit_waves", ctypes.c_int32)]


TUNING_KEYS = ("wave_threshold_16", "wave_threshold_8", "frame_groups", "crit_depth", "crit_prio",
               "crit_waves")


@dataclasses.dataclass
class Params:
    """Parameters of fse_plan (paper Section 4 defaults: d=16, rho=0.8,
    delta=0.2, gamma=0.5, 200 iterations; 64x64 DFT basis)."""
    block_w: int = 16
    block_h: int = 16
    border_d: int = 16
    fft_w: int = 64
    fft_h: int = 64
    rho: float = 0.8
    delta: float = 0.2
    gamma: float = 0.5
    iterations: int = 200
    order: int = FSE_ORDER_OPTIMIZED
    precision: int = FSE_FP32
    grid_off_x: int = 0
    grid_off_y: int = 0
    empty_fill: float = 128.0
    device_mem_budget: int = 0
    max_inflight_frames: int = 0
    flags: int = 0
    rerank_gap: float = 0.0

    def c(self) -> _Params:
        return _Params(**dataclasses.asdict(self))


_lib = None


def load():
    """Load libfse.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2207_00233_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.fse_plan.argtypes = [P(_Params), ctypes.c_void_p, P(ctypes.c_void_p)]
    lib.fse_plan.restype = ctypes.c_int32
    lib.fse_plan_destroy.argtypes = [ctypes.c_void_p]
    lib.fse_plan_destroy.restype = ctypes.c_int32
    lib.fse_conceal_image.argtypes = [ctypes.c_void_p, P(_Frame), ctypes.c_int32]
    lib.fse_conceal_image.restype = ctypes.c_int32
    lib.fse_conceal_image_noalloc.argtypes = [ctypes.c_void_p, P(_Frame), ctypes.c_int32]
    lib.fse_conceal_image_noalloc.restype = ctypes.c_int32
    lib.fse_submit.argtypes = [ctypes.c_void_p, P(_Frame), P(ctypes.c_uint64)]
    lib.fse_submit.restype = ctypes.c_int32
    lib.fse_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32]
    lib.fse_poll.restype = ctypes.c_int32
    lib.fse_schedule.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                 ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    lib.fse_schedule.restype = ctypes.c_int32
    lib.fse_schedule_refined.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    lib.fse_schedule_refined.restype = ctypes.c_int32
    lib.fse_last_call_stats.argtypes = [ctypes.c_void_p, P(_CallStats)]
    lib.fse_last_call_stats.restype = ctypes.c_int32
    lib.fse_plan_get_tuning.argtypes = [ctypes.c_void_p, P(_Tuning)]
    lib.fse_plan_get_tuning.restype = ctypes.c_int32
    lib.fse_plan_set_tuning.argtypes = [ctypes.c_void_p, P(_Tuning)]
    lib.fse_plan_set_tuning.restype = ctypes.c_int32
    lib.fse_plan_serving_stats.argtypes = [ctypes.c_void_p, P(_ServingStats)]
    lib.fse_plan_serving_stats.restype = ctypes.c_int32
    lib.fse_plan3.argtypes = [P(_Params3), ctypes.c_void_p, P(ctypes.c_void_p)]
    lib.fse_plan3.restype = ctypes.c_int32
    lib.fse_plan3_destroy.argtypes = [ctypes.c_void_p]
    lib.fse_plan3_destroy.restype = ctypes.c_int32
    lib.fse_conceal_volume.argtypes = [ctypes.c_void_p, P(_Volume)]
    lib.fse_conceal_volume.restype = ctypes.c_int32
    lib.fse_schedule3.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    lib.fse_schedule3.restype = ctypes.c_int32
    lib.fse_measure_peaks.argtypes = [P(_Peaks)]
    lib.fse_measure_peaks.restype = ctypes.c_int32
    lib.fse_strerror.argtypes = [ctypes.c_int32]
    lib.fse_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise FseError(rc, where)
    return rc


# ----------------------------------------------------------------- C-ABI calls

def fse_plan(params: Params, hip_stream: Optional[int] = None) -> "Plan":
    """Create a plan (``fse_plan``)."""
    return Plan(params, hip_stream)


def fse_schedule(lost_blocks: np.ndarray, order: int = FSE_ORDER_OPTIMIZED):
    """Processing order of a block grid (``fse_schedule``): number of waves,
    wave index per block (-1 = nothing to extrapolate), lost blocks in order."""
    lib = load()
    lb = np.ascontiguousarray(lost_blocks, dtype=np.uint8)
    hb, wb = lb.shape
    wave = np.zeros(hb * wb, np.int32)
    seq = np.zeros(max(1, hb * wb), np.int32)
    nw = _check(lib.fse_schedule(hb, wb, lb.ctypes.data, order, wave.ctypes.data,
                                 seq.ctypes.data), "fse_schedule")
    return nw, wave.reshape(hb, wb), seq[:int((lb != 0).sum())]


def fse_schedule_refined(unknown: np.ndarray, outside: int):
    """Refined processing order of a block grid (``fse_schedule_refined``):
    ``unknown`` = lost samples per block, ``outside`` = what a neighbour cell
    outside the image counts.  Returns (waves, wave index per block, lost
    blocks in order)."""
    lib = load()
    u = np.ascontiguousarray(unknown, dtype=np.int32)
    hb, wb = u.shape
    wave = np.zeros(hb * wb, np.int32)
    seq = np.zeros(max(1, hb * wb), np.int32)
    nw = _check(lib.fse_schedule_refined(hb, wb, u.ctypes.data, int(outside), wave.ctypes.data,
                                         seq.ctypes.data), "fse_schedule_refined")
    return nw, wave.reshape(hb, wb), seq[:int((u > 0).sum())]


@dataclasses.dataclass
class Result:
    out: np.ndarray                      # uint8 [H, W]
    out_f: Optional[np.ndarray] = None   # float32/float64 [H, W] unquantized
    waves: int = 0
    lost_blocks: int = 0
    max_wave_blocks: int = 0
    latency_ms: float = 0.0
    trace_block: Optional[np.ndarray] = None  # int32 [n]
    trace_wave: Optional[np.ndarray] = None   # int32 [n]
    trace_u: Optional[np.ndarray] = None      # int32 [n, K]
    trace_dc: Optional[np.ndarray] = None     # complex128 [n, K]


class _HostFrame:
    """Keeps the numpy buffers of one fse_frame alive."""

    def __init__(self, image, lost, want_float, precision, trace_cap, K):
        self.image = np.ascontiguousarray(image, dtype=np.uint8)
        self.lost = np.ascontiguousarray(lost, dtype=np.uint8)
        if self.image.shape != self.lost.shape or self.image.ndim != 2:
            raise ValueError("image and lost must be 2-D arrays of the same shape")
        H, W = self.image.shape
        self.out = np.zeros((H, W), np.uint8)
        self.of32 = (np.zeros((H, W), np.float32)
                     if want_float and precision in (FSE_FP32, FSE_FP32_RERANK, FSE_FP32_F16X3)
                     else None)
        self.of64 = np.zeros((H, W), np.float64) if want_float and precision == FSE_FP64 else None
        self.stats = _Stats()
        self.trace = None
        if trace_cap:
            self.tb = np.zeros(trace_cap, np.int32)
            self.tw = np.zeros(trace_cap, np.int32)
            self.tu = np.zeros(trace_cap * K, np.int32)
            self.tdc = np.zeros(trace_cap * K * 2, np.float64)
            P = ctypes.POINTER
            self.trace = _Trace(trace_cap, 0, self.tb.ctypes.data_as(P(ctypes.c_int32)),
                                self.tw.ctypes.data_as(P(ctypes.c_int32)),
                                self.tu.ctypes.data_as(P(ctypes.c_int32)),
                                self.tdc.ctypes.data_as(P(ctypes.c_double)))
        self.c = _Frame(self.image.ctypes.data, W, H, W, self.lost.ctypes.data, W,
                        self.out.ctypes.data, W,
                        self.of32.ctypes.data if self.of32 is not None else None,
                        self.of64.ctypes.data if self.of64 is not None else None,
                        ctypes.pointer(self.trace) if self.trace is not None else None,
                        ctypes.pointer(self.stats))

    def result(self, K) -> Result:
        r = Result(self.out, self.of32 if self.of32 is not None else self.of64,
                   self.stats.waves, self.stats.lost_blocks, self.stats.max_wave_blocks,
                   self.stats.latency_ms)
        if self.trace is not None:
            n = min(self.trace.count, len(self.tb))
            r.trace_block = self.tb[:n].copy()
            r.trace_wave = self.tw[:n].copy()
            r.trace_u = self.tu[:n * K].reshape(n, K).copy()
            d = self.tdc[:n * K * 2]
            r.trace_dc = (d[0::2] + 1j * d[1::2]).reshape(n, K)
        return r


class DeviceFrames:
    """The fse_frame array of a list of device frames (dicts as for
    Plan.conceal_device), built once so that repeated calls on the same
    buffers pass it as it is."""

    def __init__(self, frames):
        self.n = len(frames)
        self.arr = (_Frame * self.n)()
        for i, f in enumerate(frames):
            W, H = int(f["width"]), int(f["height"])
            self.arr[i] = _Frame(f["image"], W, H, W, f["lost"], W, f["out"], W,
                                 f.get("out_f32"), f.get("out_f64"), None, None)


class Plan:
    """An fse_plan handle.  Use as a context manager or call close()."""

    def __init__(self, params: Params, hip_stream: Optional[int] = None):
        self.params = params
        self._lib = load()
        h = ctypes.c_void_p()
        self._pc = params.c()
        _check(self._lib.fse_plan(ctypes.byref(self._pc), hip_stream, ctypes.byref(h)), "fse_plan")
        self.handle = h
        self._pending = {}

    def close(self):
        if self.handle:
            self._lib.fse_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    # -- fse_conceal_image ------------------------------------------------
    def fse_conceal_image(self, images: Sequence[np.ndarray], losts: Sequence[np.ndarray],
                          want_float: bool = False, trace: bool = False) -> List[Result]:
        """Conceal host images (uint8) with host loss masks, as one batch."""
        if self.params.flags & FSE_FLAG_DEVICE_PTRS:
            raise ValueError("plan expects device pointers: use conceal_device")
        K = self.params.iterations
        hf = []
        for im, ls in zip(images, losts):
            cap = 0
            if trace:
                hb = -(-(im.shape[0] + self.params.grid_off_y) // self.params.block_h)
                wb = -(-(im.shape[1] + self.params.grid_off_x) // self.params.block_w)
                cap = hb * wb
            hf.append(_HostFrame(im, ls, want_float, self.params.precision, cap, K))
        arr = (_Frame * len(hf))(*[f.c for f in hf])
        _check(self._lib.fse_conceal_image(self.handle, arr, len(hf)), "fse_conceal_image")
        return [f.result(K) for f in hf]

    def conceal_device(self, frames) -> None:
        """Conceal frames whose buffers are device memory.  ``frames`` is a list
        of dicts with integer device pointers and sizes: image, lost, out,
        width, height (strides = width), optional out_f32 / out_f64; or the
        DeviceFrames of such a list (its fse_frame array built once)."""
        if not isinstance(frames, DeviceFrames):
            frames = DeviceFrames(frames)
        _check(self._lib.fse_conceal_image(self.handle, frames.arr, frames.n), "fse_conceal_image")

    def conceal_device_noalloc(self, frames) -> None:
        """conceal_device through fse_conceal_image_noalloc: the call's device
        buffers are slices of the library's fixed scratch (nothing allocated)."""
        arr = (_Frame * len(frames))()
        for i, f in enumerate(frames):
            W, H = int(f["width"]), int(f["height"])
            arr[i] = _Frame(f["image"], W, H, W, f["lost"], W, f["out"], W,
                            f.get("out_f32"), f.get("out_f64"), None, None)
        _check(self._lib.fse_conceal_image_noalloc(self.handle, arr, len(frames)),
               "fse_conceal_image_noalloc")

    def serving_stats(self) -> dict:
        """Device memory of serving (fse_plan_serving_stats)."""
        st = _ServingStats()
        _check(self._lib.fse_plan_serving_stats(self.handle, ctypes.byref(st)),
               "fse_plan_serving_stats")
        return {k: getattr(st, k) for k, _ in _ServingStats._fields_ if k != "reserved"}

    def last_call_stats(self) -> dict:
        cs = _CallStats()
        _check(self._lib.fse_last_call_stats(self.handle, ctypes.byref(cs)), "fse_last_call_stats")
        return {k: getattr(cs, k) for k, _ in _CallStats._fields_}

    # -- fse_plan_get_tuning / fse_plan_set_tuning ------------------------------
    def get_tuning(self) -> dict:
        """Launch tuning in effect (defaults resolved)."""
        t = _Tuning()
        _check(self._lib.fse_plan_get_tuning(self.handle, ctypes.byref(t)), "fse_plan_get_tuning")
        return {k: getattr(t, k) for k in TUNING_KEYS}

    def set_tuning(self, **kw) -> None:
        """Change some of the launch tuning (keys of TUNING_KEYS); the others
        keep their values in effect."""
        bad = set(kw) - set(TUNING_KEYS)
        if bad:
            raise KeyError(f"unknown tuning keys {sorted(bad)}")
        cur = self.get_tuning()
        cur.update(kw)
        t = _Tuning(**cur)
        _check(self._lib.fse_plan_set_tuning(self.handle, ctypes.byref(t)), "fse_plan_set_tuning")

    # -- fse_submit / fse_poll ------------------------------------------------
    def fse_submit(self, image: np.ndarray, lost: np.ndarray, want_float: bool = False,
                   trace: bool = False) -> int:
        """Submit one frame for asynchronous concealment; returns a ticket."""
        K = self.params.iterations
        cap = 0
        if trace:
            hb = -(-(image.shape[0] + self.params.grid_off_y) // self.params.block_h)
            wb = -(-(image.shape[1] + self.params.grid_off_x) // self.params.block_w)
            cap = hb * wb
        f = _HostFrame(image, lost, want_float, self.params.precision, cap, K)
        t = ctypes.c_uint64()
        _check(self._lib.fse_submit(self.handle, ctypes.byref(f.c), ctypes.byref(t)), "fse_submit")
        self._pending[t.value] = f
        return t.value

    def fse_poll(self, ticket: int, timeout_us: int = 0):
        """FSE_PENDING, or the Result once the frame is done."""
        rc = self._lib.fse_poll(self.handle, ctypes.c_uint64(ticket), int(timeout_us))
        if rc == FSE_PENDING:
            return FSE_PENDING
        _check(rc, "fse_poll")
        f = self._pending.pop(ticket)
        return f.result(self.params.iterations)


def fse_conceal_image(plan: Plan, images, losts, **kw) -> List[Result]:
    return plan.fse_conceal_image(images, losts, **kw)


def fse_submit(plan: Plan, image, lost, **kw) -> int:
    return plan.fse_submit(image, lost, **kw)


def fse_poll(plan: Plan, ticket: int, timeout_us: int = 0):
    return plan.fse_poll(ticket, timeout_us)


# ------------------------------------------------------------ 3-D (video volumes)

@dataclasses.dataclass
class Params3:
    """fse_params3: three-dimensional FSE of a volume (frames x rows x
    columns) on the 8 x 32 x 32 basis grid of this build, FP64."""
    block_t: int = 1
    block_h: int = 16
    block_w: int = 16
    border_t: int = 2
    border_d: int = 8
    fft_t: int = 8
    fft_h: int = 32
    fft_w: int = 32
    rho: float = 0.8
    delta: float = 0.2
    gamma: float = 0.5
    iterations: int = 100
    order: int = FSE_ORDER_OPTIMIZED
    precision: int = FSE_FP64
    empty_fill: float = 128.0

    def c(self) -> _Params3:
        return _Params3(**dataclasses.asdict(self))


class Plan3:
    """fse_plan3 / fse_plan3_destroy / fse_conceal_volume (host arrays)."""

    def __init__(self, params: Params3, hip_stream: Optional[int] = None):
        self._lib = load()
        self.params = params
        self._pc = params.c()
        h = ctypes.c_void_p()
        _check(self._lib.fse_plan3(ctypes.byref(self._pc), hip_stream, ctypes.byref(h)),
               "fse_plan3")
        self.handle = h

    def close(self):
        if self.handle:
            self._lib.fse_plan3_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def conceal_volume(self, volume: np.ndarray, lost: np.ndarray,
                       want_float: bool = False) -> Result:
        vol = np.ascontiguousarray(volume, dtype=np.uint8)
        ls = np.ascontiguousarray(lost, dtype=np.uint8)
        if vol.ndim != 3 or ls.shape != vol.shape:
            raise ValueError("volume and lost must be frames x height x width")
        out = np.empty_like(vol)
        of = np.empty(vol.shape, np.float64) if want_float else None
        st = _Stats()
        T, H, W = vol.shape
        v = _Volume(vol.ctypes.data, ls.ctypes.data, T, H, W, out.ctypes.data,
                    of.ctypes.data if of is not None else None, ctypes.pointer(st))
        _check(self._lib.fse_conceal_volume(self.handle, ctypes.byref(v)), "fse_conceal_volume")
        return Result(out, of, st.waves, st.lost_blocks, st.max_wave_blocks, st.latency_ms)


def schedule3(lost_blocks: np.ndarray, order: int = FSE_ORDER_OPTIMIZED):
    """fse_schedule3: (waves, wave index per block, sequence) of a
    (frames, rows, columns) block grid."""
    lib = load()
    lb = np.ascontiguousarray(lost_blocks, dtype=np.uint8)
    tb, hb, wb = lb.shape
    wave = np.zeros(max(1, lb.size), np.int32)
    seq = np.zeros(max(1, lb.size), np.int32)
    nw = lib.fse_schedule3(tb, hb, wb, lb.ctypes.data, order, wave.ctypes.data, seq.ctypes.data)
    if nw < 0:
        raise FseError(nw, "fse_schedule3")
    return nw, wave[:lb.size].reshape(lb.shape), seq[:int((lb != 0).sum())]
