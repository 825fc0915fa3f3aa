"""Seeded synthetic test images.

These stand in for the paper's photographs (the 720x540 timing image of
Table 2, "Isha" of Fig. 3, the colour images of Fig. 4), which are not
available: only their shape and value statistics matter to the filter, whose
cost does not depend on the data.  All generators draw from
``numpy.random.Generator(PCG64(seed))``, return float32 arrays clipped to the
grayscale dynamic range [0, 255], and contain none of the filter's arithmetic.
Both the HIP path (through its tests and benchmark) and the FP64 oracle take
their inputs from here.
"""
from __future__ import annotations

import numpy as np

T_GRAY = 255.0


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _ramp(rng, H, W):
    u = rng.uniform(0.0, 1.0)
    y = np.arange(H, dtype=np.float64)[:, None] / max(H - 1, 1)
    x = np.arange(W, dtype=np.float64)[None, :] / max(W - 1, 1)
    return T_GRAY * (u * x + (1.0 - u) * y)


def rectangles(H: int, W: int, seed: int, n_rect: int = 12, noise: float = 10.0) -> np.ndarray:
    """Linear ramp with ``n_rect`` constant rectangles painted in order, + noise.

    Rectangle top-left corners are uniform over the image; sides are uniform in
    [W/16, W/2] (resp. H); intensities uniform in [0, 255]; noise N(0, noise^2).
    """
    rng = _rng(seed)
    img = _ramp(rng, H, W)
    for _ in range(n_rect):
        i0 = int(rng.integers(0, H))
        j0 = int(rng.integers(0, W))
        h = int(rng.uniform(H / 16.0, H / 2.0))
        w = int(rng.uniform(W / 16.0, W / 2.0))
        img[i0:i0 + max(h, 1), j0:j0 + max(w, 1)] = rng.uniform(0.0, T_GRAY)
    img = img + rng.normal(0.0, noise, size=(H, W))
    return np.clip(img, 0.0, T_GRAY).astype(np.float32)


def piecewise_smooth(H: int, W: int, seed: int, noise: float = 15.0,
                     n_shapes: int | None = None) -> np.ndarray:
    """Background ramp plus discs and rectangles with linear intensity ramps.

    K = max(4, H*W/65536) shapes (half discs, half rectangles), each of size
    U[0.02, 0.25] * min(H, W), base intensity U[0, 255] plus an in-shape ramp
    of slope up to 64/min(H, W) per pixel in a random direction; N(0, noise^2)
    noise; clipped to [0, 255].
    """
    rng = _rng(seed)
    img = _ramp(rng, H, W)
    m = min(H, W)
    K = n_shapes if n_shapes is not None else max(4, (H * W) // 65536)
    for s in range(K):
        size = rng.uniform(0.02, 0.25) * m
        ci = rng.uniform(0, H)
        cj = rng.uniform(0, W)
        base = rng.uniform(0.0, T_GRAY)
        slope = rng.uniform(0.0, 64.0 / m)
        theta = rng.uniform(0.0, 2.0 * np.pi)
        half = size / 2.0
        i0, i1 = max(0, int(ci - half)), min(H, int(ci + half) + 1)
        j0, j1 = max(0, int(cj - half)), min(W, int(cj + half) + 1)
        if i0 >= i1 or j0 >= j1:
            continue
        yy = np.arange(i0, i1, dtype=np.float64)[:, None] - ci
        xx = np.arange(j0, j1, dtype=np.float64)[None, :] - cj
        val = base + slope * (np.cos(theta) * xx + np.sin(theta) * yy)
        if s % 2 == 0:
            inside = (yy * yy + xx * xx) <= half * half
        else:
            inside = np.ones((i1 - i0, j1 - j0), dtype=bool)
        patch = img[i0:i1, j0:j1]
        patch[inside] = np.broadcast_to(val, inside.shape)[inside]
    img = img + rng.normal(0.0, noise, size=(H, W))
    return np.clip(img, 0.0, T_GRAY).astype(np.float32)


def salt(H: int, W: int, seed: int, frac: float = 0.02) -> np.ndarray:
    """Mid-gray noisy image with isolated 0/255 outliers (tiny-eta pixels)."""
    rng = _rng(seed)
    img = 128.0 + rng.normal(0.0, 8.0, size=(H, W))
    m = rng.uniform(size=(H, W)) < frac
    img[m] = np.where(rng.uniform(size=int(m.sum())) < 0.5, 0.0, T_GRAY)
    return np.clip(img, 0.0, T_GRAY).astype(np.float32)


def colour(H: int, W: int, seed: int, noise: float = 12.0) -> np.ndarray:
    """3 x H x W synthetic colour image: one piecewise-smooth structure (shared
    shapes) with per-channel intensities and independent noise, clipped to
    [0, 255]."""
    base = piecewise_smooth(H, W, seed=seed, noise=0.0)
    rng = _rng(seed + 1)
    chans = []
    for c in range(3):
        gain, off = rng.uniform(0.5, 1.0), rng.uniform(0.0, 80.0)
        ch = gain * base.astype(np.float64) + off + rng.normal(0.0, noise, size=(H, W))
        chans.append(np.clip(ch, 0.0, T_GRAY))
    return np.stack(chans).astype(np.float32)


def radius_map(H: int, W: int, seed: int, rmax: int, frac_random: float = 0.1) -> np.ndarray:
    """H x W int32 half-widths in [0, rmax] for the space-variant kernel: a
    smooth field (sum of a few wide Gaussian bumps, rescaled to [0, rmax]) with
    a fraction of pixels set to independent uniform radii, so that neighbouring
    pixels also differ sharply."""
    rng = _rng(seed)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    field = np.zeros((H, W))
    for _ in range(4):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        s = rng.uniform(0.2, 0.6) * max(H, W)
        field += rng.uniform(0.5, 1.5) * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * s * s))
    lo, hi = field.min(), field.max()
    field = (field - lo) / (hi - lo) if hi > lo else np.zeros_like(field)
    r = np.rint(field * rmax).astype(np.int32)
    m = rng.uniform(size=(H, W)) < frac_random
    r[m] = rng.integers(0, rmax + 1, size=int(m.sum()))
    return r


# --- the five workloads ------------------------------------------------------

def config_image(cfg: int) -> np.ndarray:
    """The input image of single-image workloads 1-3."""
    if cfg == 1:
        return rectangles(256, 256, seed=1)
    if cfg == 2:
        return piecewise_smooth(2048, 2048, seed=2)
    if cfg == 3:
        return piecewise_smooth(4096, 4096, seed=3)
    raise ValueError(cfg)


def diff_batch(n: int = 16, H: int = 512, W: int = 512):
    """Workload 4: n inputs (seeds 4000+i) and n SSD targets (seeds 5000+i)."""
    f = np.stack([piecewise_smooth(H, W, seed=4000 + i) for i in range(n)])
    t = np.stack([piecewise_smooth(H, W, seed=5000 + i) for i in range(n)])
    return f, t


def ragged_batch_specs(n: int = 256, seed: int = 5, lo: int = 64, hi: int = 1024):
    """Workload 5 sizes and parameters: H, W ~ U{lo..hi}, sigma_s ~ U[2,16],
    sigma_r ~ U[10,60]; image i uses seed 6000+i, its target 7000+i."""
    rng = _rng(seed)
    H = rng.integers(lo, hi + 1, size=n)
    W = rng.integers(lo, hi + 1, size=n)
    ss = rng.uniform(2.0, 16.0, size=n)
    sr = rng.uniform(10.0, 60.0, size=n)
    return [dict(H=int(H[i]), W=int(W[i]), sigma_s=float(ss[i]), sigma_r=float(sr[i]),
                 seed=6000 + i, target_seed=7000 + i) for i in range(n)]


def ragged_batch_images(specs):
    f = [piecewise_smooth(s["H"], s["W"], seed=s["seed"]) for s in specs]
    t = [piecewise_smooth(s["H"], s["W"], seed=s["target_seed"]) for s in specs]
    return f, t
