"""Seeded rectified stereo images and their 8-level pyramids.

The left image is band-limited noise; the right image is the left one warped by
a piecewise-planar disparity field plus sensor noise.  The pyramid follows the
ORB convention: level l has size (round(W/sf[l]), round(H/sf[l])) and is a
bilinear resize of level l-1.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def noise_texture(rng, H: int, W: int, blur: float = 1.5,
                  mean: float = 128.0, sd: float = 45.0) -> np.ndarray:
    n = rng.standard_normal((H, W))
    b = ndimage.gaussian_filter(n, blur, mode="reflect")
    b = (b - b.mean()) / b.std() * sd + mean
    return np.clip(np.rint(b), 0, 255).astype(np.uint8)


class DisparityField:
    """Voronoi facets, each a plane d = a + b*(x-sx) + c*(y-sy), clipped."""

    def __init__(self, rng, W: int, H: int, n_facets: int = 8,
                 d_lo: float = 2.0, d_hi: float = 60.0, slope: float = 0.03):
        self.sites = np.stack([rng.uniform(0, W, n_facets),
                               rng.uniform(0, H, n_facets)], axis=1)
        self.a = rng.uniform(d_lo, d_hi, n_facets)
        self.b = rng.uniform(-slope, slope, n_facets)
        self.c = rng.uniform(-slope, slope, n_facets)
        self.lo, self.hi = d_lo, d_hi

    def __call__(self, x, y):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        d2 = ((x[..., None] - self.sites[:, 0]) ** 2 +
              (y[..., None] - self.sites[:, 1]) ** 2)
        f = np.argmin(d2, axis=-1)
        d = (self.a[f] + self.b[f] * (x - self.sites[f, 0]) +
             self.c[f] * (y - self.sites[f, 1]))
        return np.clip(d, self.lo, self.hi)

    def right_x(self, xl, y, iters: int = 6):
        """Solve x_r + d(x_r, y) = x_l by fixed-point iteration."""
        xr = np.asarray(xl, np.float64) - self(xl, y)
        for _ in range(iters):
            xr = np.asarray(xl, np.float64) - self(xr, y)
        return xr


def right_image(rng, left: np.ndarray, field: DisparityField,
                noise_sd: float = 2.0) -> np.ndarray:
    H, W = left.shape
    xs = np.arange(W, dtype=np.float64)
    out = np.empty((H, W), np.float64)
    fresh = noise_texture(rng, H, W).astype(np.float64)
    L = left.astype(np.float64)
    for y in range(H):
        src = xs + field(xs, np.full(W, float(y)))
        x0 = np.floor(src).astype(np.int64)
        fr = src - x0
        ok = x0 + 1 <= W - 1
        x0c = np.clip(x0, 0, W - 2)
        v = L[y, x0c] * (1.0 - fr) + L[y, x0c + 1] * fr
        out[y] = np.where(ok, v, fresh[y])
    out += rng.normal(0.0, noise_sd, size=(H, W))
    return np.clip(np.rint(out), 0, 255).astype(np.uint8)


def _resize_axis(img: np.ndarray, n_out: int, axis: int) -> np.ndarray:
    n_in = img.shape[axis]
    scale = n_in / n_out
    src = (np.arange(n_out, dtype=np.float64) + 0.5) * scale - 0.5
    src = np.clip(src, 0.0, n_in - 1.0)
    i0 = np.floor(src).astype(np.int64)
    i1 = np.minimum(i0 + 1, n_in - 1)
    w = src - i0
    a = np.take(img, i0, axis=axis)
    b = np.take(img, i1, axis=axis)
    shape = [1, 1]
    shape[axis] = n_out
    w = w.reshape(shape)
    return a * (1.0 - w) + b * w


def level_sizes(W: int, H: int, sc: dict):
    inv = sc["inv_sf"]
    ws = [int(np.floor(np.float32(W) * inv[l] + np.float32(0.5))) for l in range(len(inv))]
    hs = [int(np.floor(np.float32(H) * inv[l] + np.float32(0.5))) for l in range(len(inv))]
    return ws, hs


def pyramid(img: np.ndarray, sc: dict) -> dict:
    """Pack the levels row-major, level after level, into one u8 buffer."""
    H, W = img.shape
    ws, hs = level_sizes(W, H, sc)
    levels = [img]
    for l in range(1, len(ws)):
        prev = levels[-1].astype(np.float64)
        t = _resize_axis(prev, hs[l], 0)
        t = _resize_axis(t, ws[l], 1)
        levels.append(np.clip(np.rint(t), 0, 255).astype(np.uint8))
    offs = np.zeros(len(ws), np.int64)
    acc = 0
    for l, lv in enumerate(levels):
        offs[l] = acc
        acc += lv.size
    data = np.concatenate([lv.reshape(-1) for lv in levels])
    return {"data": data, "offset": offs,
            "width": np.array(ws, np.int32), "height": np.array(hs, np.int32)}


def pyramid_level(pyr: dict, l: int) -> np.ndarray:
    o = int(pyr["offset"][l])
    w, h = int(pyr["width"][l]), int(pyr["height"][l])
    return pyr["data"][o:o + w * h].reshape(h, w)
