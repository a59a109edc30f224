"""Frame and parameter generators (seeded, synthetic).

The paper's images are not available, so frames are synthetic with the
paper's shapes (1920x1080 RGB, 8 bit):

* ``grating_frame``: per channel, a mean of 127.5 plus eight cosine gratings
  (period log-uniform in [4, 256] px, orientation uniform in [0, pi), phase
  uniform in [0, 2 pi)) of total amplitude 107.5, plus uniform noise in
  [-20, 20]; rounded half-to-even and clipped to 0..255.
* ``uniform_frames``: i.i.d. uniform [0, 1) float frames.

Parameters are plain dicts with the keys fix_x, fix_y, e0, slope, cap, block,
origin_x, origin_y (pixel-centre coordinates: (0, 0) is the centre of the
top-left pixel).
"""
from __future__ import annotations

import numpy as np

RESOLUTIONS = ((480, 640), (720, 1280), (1080, 1920), (2160, 3840))


def params_dict(fix_x, fix_y, e0, slope, cap, block=32, origin_x=0, origin_y=0):
    return dict(fix_x=float(fix_x), fix_y=float(fix_y), e0=float(e0), slope=float(slope),
                cap=float(cap), block=int(block), origin_x=int(origin_x), origin_y=int(origin_y))


def centre(h, w):
    return (w - 1) / 2.0, (h - 1) / 2.0


def central_half_fixation(rng: np.random.Generator, h: int, w: int):
    """Fixation uniform over the central half of the frame (each axis)."""
    return rng.uniform(w / 4.0, 3.0 * w / 4.0), rng.uniform(h / 4.0, 3.0 * h / 4.0)


def uniform_frames(shape, seed: int, dtype=np.float32) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(shape, dtype=np.float64).astype(dtype)


def grating_frame(h: int, w: int, c: int = 3, seed: int = 1, rng: np.random.Generator | None = None) -> np.ndarray:
    """u8 [h, w, c] frame: eight random cosine gratings per channel plus noise."""
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    ys = np.arange(h, dtype=np.float64)[:, None]
    xs = np.arange(w, dtype=np.float64)[None, :]
    out = np.empty((h, w, c), np.uint8)
    amp = 107.5 / 8.0
    for ch in range(c):
        acc = np.full((h, w), 127.5, np.float64)
        for _ in range(8):
            period = np.exp(rng.uniform(np.log(4.0), np.log(256.0)))
            theta = rng.uniform(0.0, np.pi)
            phi = rng.uniform(0.0, 2.0 * np.pi)
            kx = 2.0 * np.pi * np.cos(theta) / period
            ky = 2.0 * np.pi * np.sin(theta) / period
            # cos(kx x + ky y + phi) as a sum of two outer products
            ax = kx * xs + phi
            by = ky * ys
            acc += amp * (np.cos(by) * np.cos(ax) - np.sin(by) * np.sin(ax))
        acc += rng.uniform(-20.0, 20.0, size=(h, w))
        out[:, :, ch] = np.clip(np.rint(acc), 0, 255).astype(np.uint8)
    return out


def params_cfg1(h=256, w=256):
    """Small float frame: centre fixation, e0 32 px, slope 0.05, cap 8."""
    fx, fy = centre(h, w)
    return params_dict(fx, fy, 32.0, 0.05, 8.0)


def params_cfg2(rng: np.random.Generator | None = None, h=1080, w=1920, centred=False):
    """1080p RGB frame: fixation uniform in the central half (or the centre),
    e0 64 px, slope 0.02, cap 16."""
    if centred or rng is None:
        fx, fy = centre(h, w)
    else:
        fx, fy = central_half_fixation(rng, h, w)
    return params_dict(fx, fy, 64.0, 0.02, 16.0)


def params_cfg5(rng: np.random.Generator, h: int, w: int, e0=32.0, block=32):
    """Training-style frames: fixation uniform over the frame, slope 0.03, cap 12."""
    return params_dict(rng.uniform(0, w - 1), rng.uniform(0, h - 1), e0, 0.03, 12.0, block)


def batch_mixed(nframes: int, seed: int, resolutions=RESOLUTIONS, unique_content: int | None = None):
    """Mixed-resolution batch: resolution uniform over ``resolutions``, fixation
    uniform in the central half, slope uniform in [0.01, 0.04], cap 16, e0 64.

    Returns (frames, params): a list of u8 [h, w, 3] arrays and a list of dicts.
    ``unique_content`` bounds the number of distinct gratings drawn per
    resolution (frames of one resolution then reuse them) to keep generation
    time small for large batches.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    frames, params = [], []
    cache: dict = {}
    for i in range(nframes):
        h, w = resolutions[int(rng.integers(len(resolutions)))]
        key = (h, w)
        pool = cache.setdefault(key, [])
        if unique_content is None or len(pool) < unique_content:
            fr = grating_frame(h, w, 3, rng=np.random.Generator(np.random.PCG64(seed * 1000 + i)))
            pool.append(fr)
        else:
            fr = pool[int(rng.integers(len(pool)))]
        fx, fy = central_half_fixation(rng, h, w)
        slope = rng.uniform(0.01, 0.04)
        frames.append(fr)
        params.append(params_dict(fx, fy, 64.0, slope, 16.0))
    return frames, params
