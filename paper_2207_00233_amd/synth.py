"""Seeded synthetic inputs: 8-bit grayscale images and per-sample loss masks.

This module is shared by the tests, the benchmark and the oracle checks.  It
holds no arithmetic of the extrapolation method itself (no weighting, no
transforms, no scheduling): only random images and loss patterns with the
structure of the paper's workloads (Section 4: 16-sample square or 16-sample
wide consecutive losses on natural-image-like content).  The paper's own test
images and loss patterns are not available, so these generators stand in for
them.  Every function draws from ``numpy.random.default_rng(seed)`` (PCG64).

Conventions: an image is ``uint8[H, W]``; a loss mask is ``uint8[H, W]`` with
1 where a sample is lost.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi


def _finish(img: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


# --------------------------------------------------------------------------
# Image content
# --------------------------------------------------------------------------

def sinusoid_image(rng: np.random.Generator, height: int, width: int,
                   n_waves: int = 6, amp: Tuple[float, float] = (10.0, 40.0),
                   fmax: float = 0.25, offset: float = 128.0,
                   noise_sigma: float = 2.0) -> np.ndarray:
    """offset + sum of ``n_waves`` 2-D cosines + N(0, sigma^2), clipped, rounded.

    Horizontal and vertical frequencies are drawn independently from
    U[0, fmax] cycles/sample, amplitudes from U[amp], phases from U[0, 2pi).
    """
    y, x = np.mgrid[0:height, 0:width].astype(np.float64)
    img = np.full((height, width), offset, dtype=np.float64)
    for _ in range(n_waves):
        fx, fy = rng.uniform(0.0, fmax, size=2)
        a = rng.uniform(*amp)
        ph = rng.uniform(0.0, TWO_PI)
        img += a * np.cos(TWO_PI * (fx * x + fy * y) + ph)
    img += rng.normal(0.0, noise_sigma, size=img.shape)
    return _finish(img)


def _texture(rng: np.random.Generator, yy: np.ndarray, xx: np.ndarray,
             offset: Tuple[float, float] = (40.0, 215.0),
             amp: Tuple[float, float] = (5.0, 40.0),
             fmax: float = 0.25) -> np.ndarray:
    """One oriented sinusoidal texture evaluated at (yy, xx)."""
    off = rng.uniform(*offset)
    a = rng.uniform(*amp)
    f = rng.uniform(0.0, fmax)
    theta = rng.uniform(0.0, TWO_PI)
    ph = rng.uniform(0.0, TWO_PI)
    fx, fy = f * math.cos(theta), f * math.sin(theta)
    return (off + a * np.cos(TWO_PI * (fx * xx + fy * yy) + ph)).astype(np.float32)


def _star_polygon_mask(rng: np.random.Generator, height: int, width: int,
                       rmin: float, rmax: float):
    """Random star-shaped polygon (3..8 vertices) as (y0, x0, mask[h, w])."""
    cy = rng.uniform(0, height)
    cx = rng.uniform(0, width)
    rad = rng.uniform(rmin, rmax)
    nv = int(rng.integers(3, 9))
    ang = np.sort(rng.uniform(0.0, TWO_PI, size=nv))
    vr = rad * rng.uniform(0.4, 1.0, size=nv)
    vx = vr * np.cos(ang)
    vy = vr * np.sin(ang)
    y0 = max(0, int(math.floor(cy - rad)))
    y1 = min(height, int(math.ceil(cy + rad)) + 1)
    x0 = max(0, int(math.floor(cx - rad)))
    x1 = min(width, int(math.ceil(cx + rad)) + 1)
    if y1 <= y0 or x1 <= x0:
        return y0, x0, np.zeros((0, 0), dtype=bool)
    yy, xx = np.mgrid[y0:y1, x0:x1].astype(np.float32)
    dy = yy - np.float32(cy)
    dx = xx - np.float32(cx)
    th = np.mod(np.arctan2(dy, dx), TWO_PI).astype(np.float32)
    rho = np.sqrt(dx * dx + dy * dy)
    # Edge i runs from vertex i to vertex i+1 (cyclic); a pixel at angle th
    # lies in the sector of edge searchsorted(ang, th) - 1 (mod nv).
    seg = (np.searchsorted(ang, th, side="right") - 1) % nv
    ax, ay = vx[seg], vy[seg]
    bx, by = vx[(seg + 1) % nv], vy[(seg + 1) % nv]
    ex, ey = bx - ax, by - ay
    dxu, dyu = np.cos(th), np.sin(th)
    num = ax * ey - ay * ex
    den = dxu * ey - dyu * ex
    with np.errstate(divide="ignore", invalid="ignore"):
        rb = np.where(np.abs(den) > 1e-12, num / den, 0.0)
    return y0, x0, rho <= rb


def polygon_image(rng: np.random.Generator, height: int, width: int,
                  n_polygons: int = 20, radius: Tuple[float, float] = (20.0, 150.0),
                  noise_sigma: float = 3.0) -> np.ndarray:
    """Piecewise-smooth image: textured background, then ``n_polygons``
    textured star-shaped polygons painted later-over-earlier, plus noise."""
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float32)
    img = _texture(rng, yy, xx, offset=(90.0, 165.0))
    for _ in range(n_polygons):
        y0, x0, m = _star_polygon_mask(rng, height, width, *radius)
        if m.size == 0 or not m.any():
            # Keep the draw sequence fixed regardless of coverage.
            _texture(rng, yy[:1, :1], xx[:1, :1])
            continue
        h, w = m.shape
        tex = _texture(rng, yy[y0:y0 + h, x0:x0 + w], xx[y0:y0 + h, x0:x0 + w])
        sub = img[y0:y0 + h, x0:x0 + w]
        sub[m] = tex[m]
    img = img.astype(np.float64) + rng.normal(0.0, noise_sigma, size=img.shape)
    return _finish(img)


def drifting_frame(rng_params: np.random.Generator, height: int, width: int,
                   t: float, rng_noise: np.random.Generator) -> np.ndarray:
    """Video frame at time ``t`` (s): 4-6 sinusoids whose phases drift with
    time (phi_i + 2 pi v_i t), offset 128, plus N(0, 2^2).  ``rng_params`` is
    consumed identically for every frame of one stream (fresh copy per frame)
    so the content drifts coherently."""
    n = int(rng_params.integers(4, 7))
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float32)
    img = np.full((height, width), 128.0, dtype=np.float32)
    scale = 512.0 / max(height, width)
    for _ in range(n):
        f = rng_params.uniform(0.0, 0.25) * max(scale, 0.25)
        th = rng_params.uniform(0.0, TWO_PI)
        a = rng_params.uniform(10.0, 30.0)
        ph = rng_params.uniform(0.0, TWO_PI)
        v = rng_params.uniform(-2.0, 2.0)
        img += a * np.cos(TWO_PI * (f * math.cos(th) * xx + f * math.sin(th) * yy)
                          + ph + TWO_PI * v * t).astype(np.float32)
    img = img.astype(np.float64) + rng_noise.normal(0.0, 2.0, size=img.shape)
    return _finish(img)


# --------------------------------------------------------------------------
# Loss patterns
# --------------------------------------------------------------------------

def block_loss_mask(height: int, width: int, block: int,
                    lost_blocks: np.ndarray) -> np.ndarray:
    """Expand a boolean block grid (ceil(H/B) x ceil(W/B)) to a sample mask."""
    m = np.repeat(np.repeat(lost_blocks.astype(np.uint8), block, 0), block, 1)
    return np.ascontiguousarray(m[:height, :width])


def bernoulli_block_loss(rng: np.random.Generator, height: int, width: int,
                         block: int, p: float) -> np.ndarray:
    """Each block lost independently with probability p."""
    hb, wb = -(-height // block), -(-width // block)
    return block_loss_mask(height, width, block, rng.random((hb, wb)) < p)


def slice_loss(rng: np.random.Generator, height: int, width: int, block: int,
               frac: Tuple[float, float]) -> np.ndarray:
    """Full-width horizontal slices, 1-4 block rows tall, at uniformly random
    block rows, added until a target fraction U[frac] of block rows is lost."""
    hb, wb = -(-height // block), -(-width // block)
    target = rng.uniform(*frac)
    rows = np.zeros(hb, dtype=bool)
    guard = 0
    while rows.mean() < target and guard < 10 * hb:
        h = int(rng.integers(1, 5))
        r0 = int(rng.integers(0, hb))
        rows[r0:r0 + h] = True
        guard += 1
    grid = np.repeat(rows[:, None], wb, axis=1)
    return block_loss_mask(height, width, block, grid)


def isolated_block_loss(rng: np.random.Generator, height: int, width: int,
                        block: int, p: float) -> np.ndarray:
    """Bernoulli block losses thinned so that no two lost blocks are
    8-adjacent (the paper's isolated-loss pattern)."""
    hb, wb = -(-height // block), -(-width // block)
    cand = rng.random((hb, wb)) < p
    keep = np.zeros_like(cand)
    for i in range(hb):
        for j in range(wb):
            if cand[i, j] and not keep[max(0, i - 1):i + 2, max(0, j - 1):j + 2].any():
                keep[i, j] = True
    return block_loss_mask(height, width, block, keep)


def consecutive_loss(rng: np.random.Generator, height: int, width: int, size: int = 16,
                     runs: int = 8, length=(3, 9)) -> np.ndarray:
    """Consecutive losses of `size` samples width: horizontal and vertical runs
    of `length` cells of size x size samples on the cell grid (the paper's
    consecutive-loss pattern)."""
    hb, wb = height // size, width // size
    cells = np.zeros((hb, wb), bool)
    for _ in range(runs):
        n = int(rng.integers(length[0], length[1] + 1))
        if rng.random() < 0.5:
            i, j = int(rng.integers(0, hb)), int(rng.integers(0, max(1, wb - n + 1)))
            cells[i, j:j + n] = True
        else:
            i, j = int(rng.integers(0, max(1, hb - n + 1))), int(rng.integers(0, wb))
            cells[i:i + n, j] = True
    return block_loss_mask(height, width, size, cells)


def hole_loss(rng: np.random.Generator, height: int, width: int, n: int,
              size=(1, 12)) -> np.ndarray:
    """`n` rectangular holes of U[size] x U[size] samples at uniformly random
    positions, not aligned to any block grid (losses that leave blocks
    partially known)."""
    lost = np.zeros((height, width), np.uint8)
    for _ in range(n):
        h, w = (int(v) for v in rng.integers(size[0], size[1] + 1, 2))
        y = int(rng.integers(0, max(1, height - h + 1)))
        x = int(rng.integers(0, max(1, width - w + 1)))
        lost[y:y + h, x:x + w] = 1
    return lost


def mixed_loss(rng: np.random.Generator, height: int, width: int, size: int = 16,
               p_isolated: float = 0.12, runs: int = 6) -> np.ndarray:
    """Isolated size x size losses together with consecutive runs (the
    paper's mixed-loss pattern)."""
    iso = isolated_block_loss(rng, height, width, size, p_isolated)
    return np.maximum(iso, consecutive_loss(rng, height, width, size, runs))


# --------------------------------------------------------------------------
# The five workload recipes
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Frame:
    image: np.ndarray   # uint8 [H, W] ground truth
    lost: np.ndarray    # uint8 [H, W], 1 = lost

    @property
    def shape(self):
        return self.image.shape


def config1(seed: int = 0) -> Frame:
    """64x64 sum of 6 sinusoids + N(0, 2^2); the 16x16 block [24,40)^2 lost."""
    rng = np.random.default_rng(seed)
    img = sinusoid_image(rng, 64, 64)
    lost = np.zeros((64, 64), dtype=np.uint8)
    lost[24:40, 24:40] = 1
    return Frame(img, lost)


def config2(seed: int = 0, size: int = 512, block: int = 16, p: float = 0.25) -> Frame:
    """512x512 polygon image; 16x16 blocks lost i.i.d. with p = 0.25."""
    rng = np.random.default_rng(seed)
    img = polygon_image(rng, size, size)
    lost = bernoulli_block_loss(rng, size, size, block, p)
    return Frame(img, lost)


CONFIG3_SIZES = ((352, 288), (704, 576), (1280, 720), (1920, 1080))  # (W, H)


def config3(seed: int = 0, n_frames: int = 64, block: int = 16,
            sizes=CONFIG3_SIZES) -> List[Frame]:
    """``n_frames`` polygon images, equal counts of each size in shuffled
    order, polygon radii scaled by the image diagonal; 5-30 % slice losses."""
    rng = np.random.default_rng(seed)
    per = n_frames // len(sizes)
    order = [s for s in sizes for _ in range(per)]
    order += [sizes[i % len(sizes)] for i in range(n_frames - len(order))]
    perm = rng.permutation(len(order))
    frames = []
    ref_diag = math.hypot(512, 512)
    for idx in perm:
        w, h = order[idx]
        sc = math.hypot(w, h) / ref_diag
        img = polygon_image(rng, h, w, radius=(20.0 * sc, 150.0 * sc))
        lost = slice_loss(rng, h, w, block, (0.05, 0.30))
        frames.append(Frame(img, lost))
    return frames


SERVING_MIX = (((1280, 720), 0.3), ((1920, 1080), 0.5), ((3840, 2160), 0.2))


@dataclasses.dataclass
class Arrival:
    t: float            # arrival time (s) from stream start
    frame: Frame


def serving_stream(seed: int = 0, n_frames: int = 240, rate_hz: float = 240.0,
                   block: int = 16, mix=SERVING_MIX,
                   loss_frac=(0.02, 0.15)) -> List[Arrival]:
    """Poisson arrivals (exponential inter-arrival times, mean 1/rate) of
    drifting-texture frames of mixed resolution with slice losses."""
    rng = np.random.default_rng(seed)
    scene_seed = int(rng.integers(0, 2**31 - 1))
    sizes = [m[0] for m in mix]
    probs = np.array([m[1] for m in mix], dtype=np.float64)
    probs /= probs.sum()
    t = 0.0
    out = []
    for _ in range(n_frames):
        t += rng.exponential(1.0 / rate_hz)
        w, h = sizes[int(rng.choice(len(sizes), p=probs))]
        img = drifting_frame(np.random.default_rng(scene_seed), h, w, t, rng)
        lost = slice_loss(rng, h, w, block, loss_frac)
        out.append(Arrival(t, Frame(img, lost)))
    return out



@dataclasses.dataclass
class Volume:
    volume: np.ndarray  # uint8 [T, H, W] ground truth
    lost: np.ndarray    # uint8 [T, H, W], 1 = lost


def video_volume(seed: int = 0, frames: int = 6, height: int = 64, width: int = 80,
                 block: int = 16, p: float = 0.2, fps: float = 30.0) -> Volume:
    """``frames`` consecutive drifting-texture frames (one scene, sampled at
    ``fps``); 16 x 16 blocks of every frame lost i.i.d. with probability p,
    independently per frame, so lost blocks have known samples in the same
    block position of neighbouring frames."""
    rng = np.random.default_rng(seed)
    scene_seed = int(rng.integers(0, 2**31 - 1))
    vol = np.stack([drifting_frame(np.random.default_rng(scene_seed), height, width, z / fps, rng)
                    for z in range(frames)])
    lost = np.stack([bernoulli_block_loss(rng, height, width, block, p) for _ in range(frames)])
    return Volume(vol, lost)
