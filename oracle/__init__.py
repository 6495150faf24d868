"""FP64 CPU oracle for Frequency Selective Extrapolation (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
benchmark's CPU-baseline leg are the only permitted users.  The product path
never imports this package.  The oracle is plain C (``fse_oracle.c``) that
recomputes every projection from the spatial residual by explicit sums; it
shares nothing with the GPU implementation.

Functions (see ``fse_oracle.c`` for the readings of the paper they take):
  * :func:`block`     -- FSE over one extrapolation area (Section 2, Eq. 1-2)
  * :func:`schedule`  -- line-scan order or Algorithm 1 (Section 3, Eq. 3)
  * :func:`schedule_refined` -- the sample-count criterion Section 3 suggests
  * :func:`conceal`   -- a whole image, wave by wave, snapshot semantics
  * :func:`extract_area` -- the area and class map one block sees
  * :func:`block3`, :func:`schedule3`, :func:`conceal3`, :func:`extract_area3`
    -- the three-dimensional form for video volumes (``fse_oracle3d.c``)
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fse_oracle.c")
_SRC3 = os.path.join(_HERE, "fse_oracle3d.c")  # the three-dimensional form
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

CLS_A, CLS_R, CLS_BI, CLS_BO, CLS_OUT = 0, 1, 2, 3, 4
ORDER_OPTIMIZED, ORDER_LINESCAN, ORDER_REFINED = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over the blocks of a wave)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(_SRC), os.path.getmtime(_SRC3))):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, _SRC3, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [
        ("block_w", ctypes.c_int32), ("block_h", ctypes.c_int32),
        ("border_d", ctypes.c_int32),
        ("fft_w", ctypes.c_int32), ("fft_h", ctypes.c_int32),
        ("rho", ctypes.c_double), ("delta", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("iterations", ctypes.c_int32), ("order", ctypes.c_int32),
        ("empty_fill", ctypes.c_double),
        ("tie_largest", ctypes.c_int32),
        ("frame_off_m", ctypes.c_int32), ("frame_off_n", ctypes.c_int32),
        ("nthreads", ctypes.c_int32),
        ("grid_off_x", ctypes.c_int32), ("grid_off_y", ctypes.c_int32),
    ]


@dataclasses.dataclass
class Params:
    """FSE parameters (paper defaults from Section 4: d=16, rho=0.8,
    delta=0.2, gamma=0.5, 200 iterations)."""
    block_w: int = 16
    block_h: int = 16
    border_d: int = 16
    fft_w: int = 64
    fft_h: int = 64
    rho: float = 0.8
    delta: float = 0.2
    gamma: float = 0.5
    iterations: int = 200
    order: int = ORDER_OPTIMIZED
    empty_fill: float = 128.0
    tie_largest: int = 0
    frame_off_m: int = 0
    frame_off_n: int = 0
    nthreads: int = 0
    grid_off_x: int = 0
    grid_off_y: int = 0

    def c(self) -> _Params:
        return _Params(**dataclasses.asdict(self))

    @property
    def M(self) -> int:
        return self.block_h + 2 * self.border_d

    @property
    def N(self) -> int:
        return self.block_w + 2 * self.border_d


class _Params3(ctypes.Structure):
    _fields_ = [
        ("block_t", ctypes.c_int32), ("block_h", ctypes.c_int32), ("block_w", ctypes.c_int32),
        ("border_t", ctypes.c_int32), ("border_d", ctypes.c_int32),
        ("fft_t", ctypes.c_int32), ("fft_h", ctypes.c_int32), ("fft_w", ctypes.c_int32),
        ("rho", ctypes.c_double), ("delta", ctypes.c_double), ("gamma", ctypes.c_double),
        ("iterations", ctypes.c_int32), ("order", ctypes.c_int32),
        ("empty_fill", ctypes.c_double), ("nthreads", ctypes.c_int32),
    ]


@dataclasses.dataclass
class Params3:
    """Three-dimensional FSE of a video volume (frames x rows x columns):
    blocks of block_t x block_h x block_w samples, areas extended by border_t
    frames and border_d samples, basis grid fft_t x fft_h x fft_w."""
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
    order: int = ORDER_OPTIMIZED
    empty_fill: float = 128.0
    nthreads: int = 0

    def c(self) -> _Params3:
        return _Params3(**dataclasses.asdict(self))

    @property
    def shape(self):
        return (self.block_t + 2 * self.border_t, self.block_h + 2 * self.border_d,
                self.block_w + 2 * self.border_d)


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        lib.oracle_block.restype = ctypes.c_int
        lib.oracle_block.argtypes = [
            P(_Params), ctypes.c_int, ctypes.c_int, P(ctypes.c_double),
            P(ctypes.c_double), P(ctypes.c_uint8), P(ctypes.c_double),
            P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_double),
            P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int]
        lib.oracle_schedule.restype = ctypes.c_int
        lib.oracle_schedule.argtypes = [ctypes.c_int, ctypes.c_int,
                                        P(ctypes.c_uint8), ctypes.c_int,
                                        P(ctypes.c_int32), P(ctypes.c_int32)]
        lib.oracle_schedule_refined.restype = ctypes.c_int
        lib.oracle_schedule_refined.argtypes = [ctypes.c_int, ctypes.c_int,
                                                P(ctypes.c_int32), ctypes.c_int,
                                                P(ctypes.c_int32), P(ctypes.c_int32)]
        lib.oracle_conceal.restype = ctypes.c_int
        lib.oracle_conceal.argtypes = [
            P(_Params), ctypes.c_int, ctypes.c_int, P(ctypes.c_double),
            P(ctypes.c_uint8), P(ctypes.c_double), P(ctypes.c_int32),
            P(ctypes.c_int32), P(ctypes.c_double)]
        lib.oracle_extract_area.restype = None
        lib.oracle_extract_area.argtypes = [
            P(_Params), ctypes.c_int, ctypes.c_int, P(ctypes.c_double),
            P(ctypes.c_uint8), ctypes.c_int, ctypes.c_int, P(ctypes.c_double),
            P(ctypes.c_uint8)]
        lib.oracle3_block.restype = ctypes.c_int
        lib.oracle3_block.argtypes = [
            P(_Params3), ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_double),
            P(ctypes.c_double), P(ctypes.c_uint8), P(ctypes.c_double),
            P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_double),
            P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int]
        lib.oracle3_schedule.restype = ctypes.c_int
        lib.oracle3_schedule.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         P(ctypes.c_uint8), ctypes.c_int,
                                         P(ctypes.c_int32), P(ctypes.c_int32)]
        lib.oracle3_conceal.restype = ctypes.c_int
        lib.oracle3_conceal.argtypes = [
            P(_Params3), ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_double),
            P(ctypes.c_uint8), P(ctypes.c_double), P(ctypes.c_int32)]
        lib.oracle3_extract_area.restype = None
        lib.oracle3_extract_area.argtypes = [
            P(_Params3), ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_double),
            P(ctypes.c_uint8), ctypes.c_int, ctypes.c_int, ctypes.c_int,
            P(ctypes.c_double), P(ctypes.c_uint8)]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray], ct):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclasses.dataclass
class BlockResult:
    g: np.ndarray          # float64 [M, N], Re of the model over L
    u: np.ndarray          # int32 [K] selected indices k1*NF + k2
    dc: np.ndarray         # complex128 [K] coefficient increments
    energy: np.ndarray     # float64 [K+1] weighted residual energy
    w0: float              # sum of weights
    empty: bool            # True when L had no support
    spectrum: Optional[np.ndarray] = None  # complex128 [MF, NF]


def block(params: Params, f: np.ndarray, cls: np.ndarray,
          spec_iter: Optional[int] = None) -> BlockResult:
    """FSE over one extrapolation area (values ``f`` and classes ``cls``).
    A complex ``f`` is accepted as a test signal (the method then models
    the complex samples; the returned ``g`` is still the real part)."""
    lib = _load()
    f_im = None
    if np.iscomplexobj(f):
        f_im = np.ascontiguousarray(f.imag, dtype=np.float64)
        f = f.real
    f = np.ascontiguousarray(f, dtype=np.float64)
    cls = np.ascontiguousarray(cls, dtype=np.uint8)
    M, N = f.shape
    assert cls.shape == (M, N)
    K = params.iterations
    g = np.zeros((M, N), np.float64)
    u = np.zeros(K, np.int32)
    dc = np.zeros(2 * K, np.float64)
    e = np.zeros(K + 1, np.float64)
    w0 = np.zeros(1, np.float64)
    spec = None
    if spec_iter is not None:
        spec = np.zeros(2 * params.fft_h * params.fft_w, np.float64)
    pc = params.c()
    rc = lib.oracle_block(ctypes.byref(pc), M, N, _ptr(f, ctypes.c_double),
                          _ptr(f_im, ctypes.c_double), _ptr(cls, ctypes.c_uint8), _ptr(g, ctypes.c_double),
                          _ptr(u, ctypes.c_int32), _ptr(dc, ctypes.c_double),
                          _ptr(e, ctypes.c_double), _ptr(w0, ctypes.c_double),
                          _ptr(spec, ctypes.c_double),
                          -1 if spec_iter is None else int(spec_iter))
    sp = None
    if spec is not None:
        sp = (spec[0::2] + 1j * spec[1::2]).reshape(params.fft_h, params.fft_w)
    return BlockResult(g, u, dc[0::2] + 1j * dc[1::2], e, float(w0[0]), rc == 1, sp)


def schedule(lost_blocks: np.ndarray, order: int = ORDER_OPTIMIZED):
    """Wave index per block (-1 = nothing to extrapolate) and the processing
    sequence, for a boolean block grid."""
    lib = _load()
    lb = np.ascontiguousarray(lost_blocks, dtype=np.uint8)
    hb, wb = lb.shape
    wave = np.zeros(hb * wb, np.int32)
    seq = np.zeros(hb * wb, np.int32)
    nw = lib.oracle_schedule(hb, wb, _ptr(lb, ctypes.c_uint8), int(order),
                             _ptr(wave, ctypes.c_int32), _ptr(seq, ctypes.c_int32))
    n = int((lb != 0).sum())
    return nw, wave.reshape(hb, wb), seq[:n]


def schedule_refined(unknown: np.ndarray, outside: int):
    """Refined order of a block grid: ``unknown`` holds the lost samples of
    each block, ``outside`` what a neighbour cell outside the image counts
    (a whole block).  Returns (waves, wave index per block, sequence)."""
    lib = _load()
    u = np.ascontiguousarray(unknown, dtype=np.int32)
    hb, wb = u.shape
    wave = np.zeros(hb * wb, np.int32)
    seq = np.zeros(max(1, hb * wb), np.int32)
    nw = lib.oracle_schedule_refined(hb, wb, _ptr(u, ctypes.c_int32), int(outside),
                                     _ptr(wave, ctypes.c_int32), _ptr(seq, ctypes.c_int32))
    return nw, wave.reshape(hb, wb), seq[:int((u > 0).sum())]


@dataclasses.dataclass
class ConcealResult:
    image: np.ndarray      # float64 [H, W]
    waves: int
    wave_of: np.ndarray    # int32 [hb, wb]
    u: Optional[np.ndarray] = None    # int32 [hb, wb, K]
    dc: Optional[np.ndarray] = None   # complex128 [hb, wb, K]


def conceal(params: Params, image: np.ndarray, lost: np.ndarray,
            trace: bool = False) -> ConcealResult:
    """Conceal the lost samples of one image (values of lost samples ignored)."""
    lib = _load()
    img = np.ascontiguousarray(image, dtype=np.float64)
    ls = np.ascontiguousarray(lost, dtype=np.uint8)
    H, W = img.shape
    hb = -(-(H + params.grid_off_y) // params.block_h)
    wb = -(-(W + params.grid_off_x) // params.block_w)
    out = np.zeros((H, W), np.float64)
    wave = np.zeros(hb * wb, np.int32)
    K = params.iterations
    tu = np.zeros(hb * wb * K, np.int32) if trace else None
    tdc = np.zeros(hb * wb * 2 * K, np.float64) if trace else None
    pc = params.c()
    nw = lib.oracle_conceal(ctypes.byref(pc), H, W, _ptr(img, ctypes.c_double),
                            _ptr(ls, ctypes.c_uint8), _ptr(out, ctypes.c_double),
                            _ptr(wave, ctypes.c_int32), _ptr(tu, ctypes.c_int32),
                            _ptr(tdc, ctypes.c_double))
    if nw < 0:
        raise ValueError("invalid oracle parameters")
    res = ConcealResult(out, nw, wave.reshape(hb, wb))
    if trace:
        res.u = tu.reshape(hb, wb, K)
        res.dc = (tdc[0::2] + 1j * tdc[1::2]).reshape(hb, wb, K)
    return res


def extract_area(params: Params, image: np.ndarray, state: np.ndarray,
                 bi: int, bj: int):
    """Values and classes of the area of block (bi, bj) given a working image
    and a state map (0 known, 1 pending, 2 reconstructed)."""
    lib = _load()
    img = np.ascontiguousarray(image, dtype=np.float64)
    st = np.ascontiguousarray(state, dtype=np.uint8)
    H, W = img.shape
    f = np.zeros((params.M, params.N), np.float64)
    cls = np.zeros((params.M, params.N), np.uint8)
    pc = params.c()
    lib.oracle_extract_area(ctypes.byref(pc), H, W, _ptr(img, ctypes.c_double),
                            _ptr(st, ctypes.c_uint8), int(bi), int(bj),
                            _ptr(f, ctypes.c_double), _ptr(cls, ctypes.c_uint8))
    return f, cls


# ------------------------------------------------------------------ 3-D form

def block3(params: Params3, f: np.ndarray, cls: np.ndarray,
           spec_iter: Optional[int] = None) -> BlockResult:
    """Three-dimensional FSE over one area (values ``f`` and classes ``cls``,
    both Mt x M x N); a complex ``f`` is accepted as a test signal."""
    lib = _load()
    f_im = None
    if np.iscomplexobj(f):
        f_im = np.ascontiguousarray(f.imag, dtype=np.float64)
        f = f.real
    f = np.ascontiguousarray(f, dtype=np.float64)
    cls = np.ascontiguousarray(cls, dtype=np.uint8)
    Mt, M, N = f.shape
    assert cls.shape == f.shape
    K = params.iterations
    F = params.fft_t * params.fft_h * params.fft_w
    g = np.zeros(f.shape, np.float64)
    u = np.zeros(K, np.int32)
    dc = np.zeros(2 * K, np.float64)
    e = np.zeros(K + 1, np.float64)
    w0 = np.zeros(1, np.float64)
    spec = np.zeros(2 * F, np.float64) if spec_iter is not None else None
    pc = params.c()
    rc = lib.oracle3_block(ctypes.byref(pc), Mt, M, N, _ptr(f, ctypes.c_double),
                           _ptr(f_im, ctypes.c_double), _ptr(cls, ctypes.c_uint8),
                           _ptr(g, ctypes.c_double), _ptr(u, ctypes.c_int32),
                           _ptr(dc, ctypes.c_double), _ptr(e, ctypes.c_double),
                           _ptr(w0, ctypes.c_double), _ptr(spec, ctypes.c_double),
                           -1 if spec_iter is None else int(spec_iter))
    sp = None
    if spec is not None:
        sp = (spec[0::2] + 1j * spec[1::2]).reshape(params.fft_t, params.fft_h, params.fft_w)
    return BlockResult(g, u, dc[0::2] + 1j * dc[1::2], e, float(w0[0]), rc == 1, sp)


def schedule3(lost_blocks: np.ndarray, order: int = ORDER_OPTIMIZED):
    """Processing order of a (frames, rows, columns) block grid over the
    26-neighbourhood: (waves, wave index per block, sequence)."""
    lib = _load()
    lb = np.ascontiguousarray(lost_blocks, dtype=np.uint8)
    tb, hb, wb = lb.shape
    wave = np.zeros(lb.size, np.int32)
    seq = np.zeros(max(1, lb.size), np.int32)
    nw = lib.oracle3_schedule(tb, hb, wb, _ptr(lb, ctypes.c_uint8), int(order),
                              _ptr(wave, ctypes.c_int32), _ptr(seq, ctypes.c_int32))
    return nw, wave.reshape(tb, hb, wb), seq[:int((lb != 0).sum())]


@dataclasses.dataclass
class Conceal3Result:
    volume: np.ndarray     # float64 [T, H, W]
    waves: int
    wave_of: np.ndarray    # int32 [tb, hb, wb]


def conceal3(params: Params3, volume: np.ndarray, lost: np.ndarray) -> Conceal3Result:
    """Conceal the lost samples of a volume (values of lost samples ignored)."""
    lib = _load()
    vol = np.ascontiguousarray(volume, dtype=np.float64)
    ls = np.ascontiguousarray(lost, dtype=np.uint8)
    T, H, W = vol.shape
    tb, hb, wb = -(-T // params.block_t), -(-H // params.block_h), -(-W // params.block_w)
    out = np.zeros(vol.shape, np.float64)
    wave = np.zeros(tb * hb * wb, np.int32)
    pc = params.c()
    nw = lib.oracle3_conceal(ctypes.byref(pc), T, H, W, _ptr(vol, ctypes.c_double),
                             _ptr(ls, ctypes.c_uint8), _ptr(out, ctypes.c_double),
                             _ptr(wave, ctypes.c_int32))
    if nw < 0:
        raise ValueError("invalid oracle parameters")
    return Conceal3Result(out, nw, wave.reshape(tb, hb, wb))


def extract_area3(params: Params3, volume: np.ndarray, state: np.ndarray,
                  bt: int, bi: int, bj: int):
    """Values and classes of the 3-D area of block (bt, bi, bj)."""
    lib = _load()
    vol = np.ascontiguousarray(volume, dtype=np.float64)
    st = np.ascontiguousarray(state, dtype=np.uint8)
    T, H, W = vol.shape
    f = np.zeros(params.shape, np.float64)
    cls = np.zeros(params.shape, np.uint8)
    pc = params.c()
    lib.oracle3_extract_area(ctypes.byref(pc), T, H, W, _ptr(vol, ctypes.c_double),
                             _ptr(st, ctypes.c_uint8), int(bt), int(bi), int(bj),
                             _ptr(f, ctypes.c_double), _ptr(cls, ctypes.c_uint8))
    return f, cls
