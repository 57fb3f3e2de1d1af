"""Seeded 8-bit grayscale test frames.

Recipe (one frame, ``rng = numpy.random.default_rng(seed)``):

1. base value 128 plus the sum of 8 plane waves
   ``a*sin(2*pi*(x*cos(theta) + y*sin(theta))/T + phi)`` with
   ``a ~ U[5,40]``, ``T ~ U[4,64]`` pixels, ``theta ~ U[0,pi)``,
   ``phi ~ U[0,2*pi)``;
2. 6 filled polygons painted in order (later ones overwrite earlier ones),
   each of constant gray ``U[0,255]``, with ``U{3..8}`` vertices placed at
   sorted random angles around a uniformly drawn centre, at radii
   ``U[0.05,0.25]*min(H,W)`` (star-shaped, hence simple);
3. additive Gaussian noise with sigma 2;
4. round half to even, clip to [0,255], cast to uint8.
"""
import numpy as np


def _fill_polygon(img, ys, xs, value):
    """Paint the even-odd interior of a closed polygon (vertex arrays ys, xs)
    into ``img`` in place; pixel (y, x) is sampled at its integer position."""
    H, W = img.shape
    y_lo = max(int(np.floor(ys.min())), 0)
    y_hi = min(int(np.ceil(ys.max())), H - 1)
    x_lo = max(int(np.floor(xs.min())), 0)
    x_hi = min(int(np.ceil(xs.max())), W - 1)
    if y_lo > y_hi or x_lo > x_hi:
        return
    py = np.arange(y_lo, y_hi + 1, dtype=np.float64)[:, None]
    px = np.arange(x_lo, x_hi + 1, dtype=np.float64)[None, :]
    inside = np.zeros((y_hi - y_lo + 1, x_hi - x_lo + 1), dtype=bool)
    n = len(ys)
    for i in range(n):
        y0, x0 = ys[i], xs[i]
        y1, x1 = ys[(i + 1) % n], xs[(i + 1) % n]
        if y0 == y1:
            continue
        # edge crosses the horizontal ray through py to the right of px
        spans = (py >= min(y0, y1)) & (py < max(y0, y1))
        x_at = x0 + (py - y0) * (x1 - x0) / (y1 - y0)
        inside ^= spans & (px < x_at)
    img[y_lo:y_hi + 1, x_lo:x_hi + 1][inside] = value


def synthetic_image(height, width, seed, n_waves=8, n_polygons=6, noise_sigma=2.0):
    """Return one ``uint8[height][width]`` frame drawn from ``seed``."""
    rng = np.random.default_rng(seed)
    y = np.arange(height, dtype=np.float64)[:, None]
    x = np.arange(width, dtype=np.float64)[None, :]
    img = np.full((height, width), 128.0)
    for _ in range(n_waves):
        a = rng.uniform(5.0, 40.0)
        period = rng.uniform(4.0, 64.0)
        theta = rng.uniform(0.0, np.pi)
        phase = rng.uniform(0.0, 2.0 * np.pi)
        img += a * np.sin(2.0 * np.pi * (x * np.cos(theta) + y * np.sin(theta)) / period + phase)
    short = min(height, width)
    for _ in range(n_polygons):
        gray = rng.uniform(0.0, 255.0)
        nv = int(rng.integers(3, 9))
        cy = rng.uniform(0.0, height)
        cx = rng.uniform(0.0, width)
        ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, size=nv))
        rad = rng.uniform(0.05, 0.25, size=nv) * short
        _fill_polygon(img, cy + rad * np.sin(ang), cx + rad * np.cos(ang), gray)
    img += rng.normal(0.0, noise_sigma, size=img.shape)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def synthetic_frames(height, width, seeds):
    """Stack of independent frames, one per seed: ``uint8[len(seeds)][H][W]``."""
    return np.stack([synthetic_image(height, width, s) for s in seeds])


def synthetic_clip(height, width, n_frames, seed, max_shift=3):
    """A video clip: one synthetic image of a larger canvas, viewed through a
    window that moves by a random integer translation of up to +-max_shift
    pixels per frame (clamped to the canvas): ``uint8[n_frames][H][W]``."""
    rng = np.random.default_rng(seed + 2 * 10 ** 6)
    pad = max_shift * n_frames
    canvas = synthetic_image(height + 2 * pad, width + 2 * pad, seed)
    y = x = pad
    out = np.empty((n_frames, height, width), dtype=np.uint8)
    for f in range(n_frames):
        out[f] = canvas[y:y + height, x:x + width]
        y = int(np.clip(y + rng.integers(-max_shift, max_shift + 1), 0, 2 * pad))
        x = int(np.clip(x + rng.integers(-max_shift, max_shift + 1), 0, 2 * pad))
    return out
