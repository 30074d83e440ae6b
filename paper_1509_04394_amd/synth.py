"""Seeded synthetic high-speed-video generator.

The paper evaluates on high-speed facial video (600-1000 frames/s, frames of
192x432 and 800x600 pixels; Sec. I and Sec. VII-A).  That footage is not
available, so every workload here is synthetic video of the same shape and
character: a smooth static background, moving bright blobs (the tracked
features) and sensor noise, quantised to uint8.

This module only makes inputs.  It holds none of the arithmetic of the kernel
chain, and both the GPU path and the CPU reference consume what it produces.

Recipe (all draws from numpy PCG64 seeded by ``seed``):
  * background: a uniform 6x4 control grid (6 along x, 4 along y) upsampled by a
    bicubic spline to W x H, min-max rescaled to [40, 200]; static for the clip;
    an independent grid per channel for RGB;
  * 20 Gaussian blobs, sigma 3 px, amplitude +60, centre per axis
    p(t) = p0 + v t + A sin(w t + phi), p0 ~ U(frame), |v| <= 1 px/frame,
    A ~ U[2, 10] px, w ~ U[0.02, 0.2], phi ~ U[0, 2 pi); positions wrap on the
    frame torus so blobs stay in view for long clips;
  * additive N(0, 4^2) noise, iid per pixel (and per channel); the noise of
    frame t comes from its own stream seeded by (seed, t), so any frame range
    can be regenerated on its own;
  * rint (half-to-even), clip to [0, 255], uint8.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
from scipy.interpolate import RectBivariateSpline

N_BLOBS = 20
BLOB_SIGMA = 3.0
BLOB_AMP = 60.0
NOISE_SIGMA = 4.0
BG_LO, BG_HI = 40.0, 200.0
_BLOB_R = 12  # draw window half-size (4 sigma)


class VideoSpec:
    """Per-clip draws: background planes and blob trajectories."""

    def __init__(self, width: int, height: int, seed: int, channels: int = 1):
        if width <= 0 or height <= 0:
            raise ValueError("frame size must be positive")
        self.W, self.H, self.C, self.seed = int(width), int(height), int(channels), int(seed)
        rng = np.random.default_rng(seed)
        xs = np.linspace(0.0, self.W - 1.0, 6)
        ys = np.linspace(0.0, self.H - 1.0, 4)
        px = np.arange(self.W, dtype=np.float64)
        py = np.arange(self.H, dtype=np.float64)
        planes = []
        for _ in range(self.C):
            grid = rng.uniform(0.0, 1.0, size=(4, 6))
            spl = RectBivariateSpline(ys, xs, grid, kx=3, ky=3)
            bg = spl(py, px)
            lo, hi = bg.min(), bg.max()
            bg = (bg - lo) / max(hi - lo, 1e-12) * (BG_HI - BG_LO) + BG_LO
            planes.append(bg.astype(np.float32))
        self.background = np.stack(planes, axis=-1)  # [H][W][C]
        self.p0 = np.stack([rng.uniform(0, self.W, N_BLOBS), rng.uniform(0, self.H, N_BLOBS)], 1)
        speed = rng.uniform(0.0, 1.0, N_BLOBS)
        ang = rng.uniform(0.0, 2 * np.pi, N_BLOBS)
        self.v = np.stack([speed * np.cos(ang), speed * np.sin(ang)], 1)
        self.amp = rng.uniform(2.0, 10.0, (N_BLOBS, 2))
        self.omega = rng.uniform(0.02, 0.2, (N_BLOBS, 2))
        self.phi = rng.uniform(0.0, 2 * np.pi, (N_BLOBS, 2))
        off = np.arange(-_BLOB_R, _BLOB_R + 1, dtype=np.float64)
        self._off = off

    def centres(self, t: int) -> np.ndarray:
        p = self.p0 + self.v * t + self.amp * np.sin(self.omega * t + self.phi)
        return np.mod(p, [self.W, self.H])

    def frame(self, t: int) -> np.ndarray:
        """Frame t as uint8 [H][W][C]."""
        f = self.background.copy()
        W, H = self.W, self.H
        for cx, cy in self.centres(t):
            ix = int(np.floor(cx))
            iy = int(np.floor(cy))
            xs = ix + np.arange(-_BLOB_R, _BLOB_R + 2)
            ys = iy + np.arange(-_BLOB_R, _BLOB_R + 2)
            gx = np.exp(-((xs - cx) ** 2) / (2 * BLOB_SIGMA ** 2))
            gy = np.exp(-((ys - cy) ** 2) / (2 * BLOB_SIGMA ** 2))
            patch = (BLOB_AMP * np.outer(gy, gx)).astype(np.float32)
            # wrap the patch on the torus
            np.add.at(f, (np.mod(ys, H)[:, None], np.mod(xs, W)[None, :]), patch[:, :, None])
        nrng = np.random.default_rng([self.seed, t])
        f += NOISE_SIGMA * nrng.standard_normal(f.shape, dtype=np.float32)
        np.rint(f, out=f)
        np.clip(f, 0, 255, out=f)
        return f.astype(np.uint8)


def video(width: int, height: int, frames: int, seed: int, rgb: bool = False,
          t0: int = 0, out: np.ndarray | None = None, workers: int | None = None) -> np.ndarray:
    """Frames [t0, t0+frames) of the clip.

    Gray: uint8 [T][H][W].  RGB: uint8 [T][H][W][3] (interleaved).  Frames are
    independent draws, so they are made in parallel threads; the result does
    not depend on ``workers``.
    """
    spec = VideoSpec(width, height, seed, 3 if rgb else 1)
    shape = (frames, height, width, 3) if rgb else (frames, height, width)
    if out is None:
        out = np.empty(shape, np.uint8)

    def one(i):
        fr = spec.frame(t0 + i)
        out[i] = fr if rgb else fr[:, :, 0]

    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers <= 1 or frames < 4:
        for i in range(frames):
            one(i)
    else:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(one, range(frames)))
    return out


def field_f32(shape, seed: int, lo: float, hi: float, smooth: bool = True) -> np.ndarray:
    """Seeded float32 field for feeding a stage that takes float input.

    Values are uniform in [lo, hi]; with ``smooth`` a 3-tap running mean along
    each spatial axis gives neighbouring pixels correlated values.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(lo, hi, size=shape)
    if smooth:
        a = (a + np.roll(a, 1, -1) + np.roll(a, -1, -1)) / 3.0
        a = (a + np.roll(a, 1, -2) + np.roll(a, -1, -2)) / 3.0
    return a.astype(np.float32)


def response_field(shape, seed: int, thr: float, n_peaks_per_frame: int = 12) -> np.ndarray:
    """Seeded float32 corner-response-like field [T][H][W]: a mostly sub-threshold
    background with isolated peaks well above ``thr`` and a few plateaus (equal
    neighbouring maxima), for exercising threshold / suppression decisions."""
    rng = np.random.default_rng(seed)
    T, H, W = shape
    a = rng.uniform(-0.5 * thr, 0.9 * thr, size=shape)
    for t in range(T):
        for _ in range(n_peaks_per_frame):
            y = int(rng.integers(0, H)); x = int(rng.integers(0, W))
            a[t, y, x] = rng.uniform(1.5 * thr, 20 * thr)
        # plateau: two equal neighbouring maxima
        y = int(rng.integers(0, H)); x = int(rng.integers(0, max(W - 1, 1)))
        v = 30 * thr
        a[t, y, x] = v
        if x + 1 < W:
            a[t, y, x + 1] = v
    return a.astype(np.float32)


def ramp(width: int, height: int, frames: int, a: float, b: float, c: float) -> np.ndarray:
    """uint8 linear ramp a*x + b*y + c (x along width), for closed-form checks."""
    x = np.arange(width)[None, :]
    y = np.arange(height)[:, None]
    f = a * x + b * y + c
    if f.min() < 0 or f.max() > 255 or np.any(f != np.round(f)):
        raise ValueError("ramp must be integral in [0, 255]")
    return np.broadcast_to(f.astype(np.uint8), (frames, height, width)).copy()


POINT_KINDS = ("affine", "abs", "square", "sqrtabs", "clamp")


def random_chain(seed: int, length: int | None = None, max_r: int = 3):
    """A random chain of generic single-channel stages, for planner and cost
    model workloads.

    Recipe (numpy PCG64 seeded by ``seed``): length ~ U{4..16} unless given;
    each stage's class uniform over {stencil, point, box}:
      * stencil: radius r ~ U{0..max_r} on both axes, weights N(0, 1) scaled so
        that their absolute values sum to 1;
      * point: kind uniform over POINT_KINDS; affine a = +-U[0.5, 2],
        b ~ U[-20, 20]; clamp lo ~ U[-50, 50], hi = lo + U[10, 200];
      * box: radius r ~ U{1..max_r} on both axes.
    Every number is rounded to float32 here, so the values any consumer sees
    are exactly representable in single precision.  Stages are tuples
    ("stencil", rx, ry, w[2ry+1][2rx+1]), ("point", kind, a, b), ("box", rx, ry).
    """
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 17)) if length is None else int(length)
    f32 = lambda v: float(np.float32(v))
    out = []
    for _ in range(n):
        cls = int(rng.integers(0, 3))
        if cls == 0:
            r = int(rng.integers(0, max_r + 1))
            w = rng.standard_normal((2 * r + 1, 2 * r + 1))
            w = (w / np.abs(w).sum()).astype(np.float32)
            out.append(("stencil", r, r, w))
        elif cls == 1:
            kind = POINT_KINDS[int(rng.integers(0, len(POINT_KINDS)))]
            if kind == "affine":
                a = rng.uniform(0.5, 2.0) * (1 if rng.random() < 0.5 else -1)
                out.append(("point", kind, f32(a), f32(rng.uniform(-20, 20))))
            elif kind == "clamp":
                lo = f32(rng.uniform(-50, 50))
                out.append(("point", kind, lo, f32(lo + rng.uniform(10, 200))))
            else:
                out.append(("point", kind, 0.0, 0.0))
        else:
            r = int(rng.integers(1, max_r + 1))
            out.append(("box", r, r))
    return out


BATCH_SIZES = [(192, 432), (320, 240), (640, 480), (800, 600)]


def batch_shapes(seed: int, n: int, t_lo: int = 50, t_hi: int = 1000):
    """(W, H, T) of n clips of a batch: frame size uniform over BATCH_SIZES,
    frame count uniform in [t_lo, t_hi]; clip i's video uses seed 4000 + i."""
    rng = np.random.default_rng(seed)
    return [(*BATCH_SIZES[int(rng.integers(0, len(BATCH_SIZES)))], int(rng.integers(t_lo, t_hi + 1)))
            for _ in range(n)]
