"""Seeded synthetic space-time feature volumes.

The method (Sec. 3) takes per-pixel feature maps S (unary) and F (pairwise)
over a T x H x W clip; in the paper's experiments S is an input soft
segmentation (Sec. 5, experimental setup).  No dataset is used here: these
generators draw clips with the same structure -- one salient moving object on
a zero background, a few static distractor blobs, additive Gaussian noise,
values clipped to [0, 1].

This module holds no arithmetic of the method itself.  It is the only code
shared by the oracle-side tests and the GPU path's tests and benchmark.

Recipes (all numpy PCG64, fully determined by the seed):

* ``tiny_clip``   8x64x96: object ellipse at 0.8 whose centre drifts by
  N(0, 1.5 px) per frame, 2 static discs at 0.4, noise sigma 0.1.
* ``full_clip``  70x480x854: object ellipse at 0.8 under a cumulative random
  affine motion per frame (translation N(0, 2 px), rotation N(0, 2 deg),
  scale 1 + N(0, 0.01)), 3 static discs at 0.4, noise sigma 0.15.
* ``make_clip``   the general form both are built on.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["make_clip", "tiny_clip", "full_clip", "ragged_shapes", "random_vector",
           "feature_channels"]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def make_clip(T: int, H: int, W: int, *, seed: int, n_blobs: int = 3,
              noise_sigma: float = 0.15, motion: str = "affine",
              object_value: float = 0.8, blob_value: float = 0.4,
              dtype=np.float32) -> np.ndarray:
    """Return a (T, H, W) array of soft-segmentation-like features in [0, 1].

    ``motion`` is ``"drift"`` (centre random walk, sigma 1.5 px) or
    ``"affine"`` (cumulative translation / rotation / scale per frame).
    """
    if T < 1 or H < 1 or W < 1:
        raise ValueError("T, H, W must be >= 1")
    if motion not in ("drift", "affine"):
        raise ValueError("motion must be 'drift' or 'affine'")
    rng = _rng(seed)
    a0 = 0.18 * H          # vertical semi-axis of the object
    b0 = 0.12 * W          # horizontal semi-axis of the object
    cy = rng.uniform(0.25 * H, 0.75 * H)
    cx = rng.uniform(0.25 * W, 0.75 * W)
    theta = 0.0
    scale = 1.0

    # Static distractor discs, placed away from the object's start position.
    blobs = []
    for _ in range(n_blobs):
        rad = rng.uniform(0.05, 0.08) * H
        for _attempt in range(64):
            by = rng.uniform(rad, max(rad, H - rad))
            bx = rng.uniform(rad, max(rad, W - rad))
            if math.hypot((by - cy) / max(a0, 1e-9), (bx - cx) / max(b0, 1e-9)) > 1.6:
                break
        blobs.append((by, bx, rad))

    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64),
                         np.arange(W, dtype=np.float64), indexing="ij")
    base = np.zeros((H, W), dtype=np.float64)
    for by, bx, rad in blobs:
        base[(yy - by) ** 2 + (xx - bx) ** 2 <= rad * rad] = blob_value

    out = np.empty((T, H, W), dtype=dtype)
    for t in range(T):
        if t > 0:
            if motion == "drift":
                cy += rng.normal(0.0, 1.5)
                cx += rng.normal(0.0, 1.5)
            else:
                cy += rng.normal(0.0, 2.0)
                cx += rng.normal(0.0, 2.0)
                theta += math.radians(rng.normal(0.0, 2.0))
                scale *= 1.0 + rng.normal(0.0, 0.01)
            # keep the object centre inside the central region of the frame
            cy = min(max(cy, 0.2 * H), 0.8 * H)
            cx = min(max(cx, 0.2 * W), 0.8 * W)
        frame = base.copy()
        c, s = math.cos(theta), math.sin(theta)
        dy, dx = yy - cy, xx - cx
        u = (c * dy + s * dx) / max(a0 * scale, 1e-9)
        v = (-s * dy + c * dx) / max(b0 * scale, 1e-9)
        frame[u * u + v * v <= 1.0] = object_value
        frame += rng.normal(0.0, noise_sigma, size=(H, W))
        np.clip(frame, 0.0, 1.0, out=frame)
        out[t] = frame.astype(dtype)
    return out


def tiny_clip(seed: int = 0, dtype=np.float64) -> np.ndarray:
    """8 x 64 x 96 clip: drifting ellipse, 2 distractor discs, noise 0.1."""
    return make_clip(8, 64, 96, seed=seed, n_blobs=2, noise_sigma=0.1,
                     motion="drift", dtype=dtype)


def full_clip(seed: int = 1, dtype=np.float32, T: int = 70, H: int = 480,
              W: int = 854) -> np.ndarray:
    """70 x 480 x 854 clip: affine-moving ellipse, 3 discs, noise 0.15."""
    return make_clip(T, H, W, seed=seed, n_blobs=3, noise_sigma=0.15,
                     motion="affine", dtype=dtype)


def feature_channels(T: int, H: int, W: int, *, seed: int, n_blobs: int = 3,
                     noise_sigma: float = 0.15, motion: str = "affine",
                     dtype=np.float32) -> np.ndarray:
    """Two pairwise feature channels (2, T, H, W) for the multi-channel form:
    channel 0 is the clip itself (object, distractors, noise), channel 1 a
    motion-like map of the same scene -- the moving object at 1.0 with the
    same trajectory, no static distractors, light noise (sigma 0.05)."""
    a = make_clip(T, H, W, seed=seed, n_blobs=n_blobs, noise_sigma=noise_sigma, motion=motion,
                  dtype=dtype)
    b = make_clip(T, H, W, seed=seed, n_blobs=n_blobs, noise_sigma=0.05, motion=motion,
                  object_value=1.0, blob_value=0.0, dtype=dtype)
    return np.stack([a, b])


def ragged_shapes(n: int, seed: int = 3):
    """Shapes of ``n`` clips of uneven size: frames uniform in 20..100,
    resolution drawn from {240x427, 360x640, 480x854}."""
    rng = _rng(seed)
    res = [(240, 427), (360, 640), (480, 854)]
    out = []
    for _ in range(n):
        T = int(rng.integers(20, 101))
        H, W = res[int(rng.integers(0, 3))]
        out.append((T, H, W))
    return out


def random_vector(shape, seed: int, signed: bool = False, dtype=np.float64) -> np.ndarray:
    """Seeded random test vector: U[0,1) or, if ``signed``, U[-1,1)."""
    rng = _rng(seed)
    x = rng.random(size=shape)
    if signed:
        x = 2.0 * x - 1.0
    return x.astype(dtype)
