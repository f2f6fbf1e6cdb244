"""Adaptive masked training (Sec. 3.3, "Adaptive Masked Training"; values in the appendix's implementation
details), FP64 (oracle; test only).

The paper splits the Gaussians into static and dynamic ones by a threshold t_d on the norm of the score d_t
(Eq. 9), renders the dynamic ones for each training view to find the dynamic image regions, dilates that
image mask with a 48 x 48 kernel, and for a fraction of a frame's iterations renders and backpropagates
only there.  Readings taken here where the text leaves a choice open:

* dynamic: ||d_i|| / V > t_d, with d the view sum of Eq. 9's bracket (so d / V is Eq. 9's mean) taken in
  normalised device coordinates, the units of the viewspace gradient of the 3D-GS rasterizer the method builds
  on (pixel gradients times W/2 and H/2), t_d = 0.001;
* the image mask of a view: the pixels the dynamic-only render reaches (T_final < 1), i.e. where some dynamic
  splat has alpha >= 1/255;
* dilation by a k x k box (k = 48): pixel (x, y) is set if the mask has a set pixel in
  [x - k//2, x + k - 1 - k//2] x [y - k//2, y + k - 1 - k//2] (the kernel's anchor at offset k//2);
* rendering is skipped per tile: a tile is rendered if its dilated mask has a set pixel;
* the masked loss is the L1 over the dilated-mask pixels at the full image's normalisation 1/(3HW), with a
  zero image gradient elsewhere;
* schedule: the first ceil(f K) of a frame's K iterations are masked (f = 0.30 for N3DV, 0.65 for Immersive),
  the rest use the full image.

Pinned by closed forms and invariants (tests/test_oracle_mask.py): the dilation of one pixel is the k x k
square at the stated offsets, clipped at the border; dilation distributes over union; an all-ones mask gives
the plain L1; a single dynamic splat's mask is its alpha >= 1/255 ellipse.
"""
from __future__ import annotations

import math

import numpy as np

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99


def dynamic_flags(d: np.ndarray, n_views: int, width: int, height: int, t_d: float = 1e-3) -> np.ndarray:
    """d [2][N] (view sum of Eq. 9's bracket, in pixels) -> bool [N]: the norm of the view mean in normalised
    device coordinates, ||(dx W/2, dy H/2)|| / V, exceeds t_d."""
    d = np.asarray(d, np.float64)
    x = d[0] * ((width / 2.0) / n_views)
    y = d[1] * ((height / 2.0) / n_views)
    return np.sqrt(x * x + y * y) > t_d


def footprint(xy, conic, opacity, width: int, height: int) -> np.ndarray:
    """Pixels (centres at +0.5) where one splat reaches alpha = min(0.99, o exp(-q/2)) >= 1/255 -> bool [H][W]."""
    X, Y = np.meshgrid(np.arange(width) + 0.5, np.arange(height) + 0.5)
    dx, dy = X - float(xy[0]), Y - float(xy[1])
    A, B, C = (float(c) for c in conic)
    q = A * dx * dx + 2.0 * B * dx * dy + C * dy * dy
    return np.minimum(ALPHA_MAX, float(opacity) * np.exp(-0.5 * q)) >= ALPHA_MIN


def dynamic_mask(T_final_dynamic: np.ndarray) -> np.ndarray:
    """Image mask from the render of the dynamic Gaussians alone: the pixels it reaches (T_final < 1)."""
    return np.asarray(T_final_dynamic, np.float64) < 1.0


def dilate(mask: np.ndarray, k: int = 48) -> np.ndarray:
    """k x k box dilation with offsets [-(k//2), k - 1 - k//2] on both axes, clipped to the image."""
    m = np.asarray(mask, bool)
    H, W = m.shape
    lo, hi = -(k // 2), k - 1 - k // 2
    out = np.zeros_like(m)
    for y in range(H):
        for x in range(W):
            y0, y1 = max(0, y + lo), min(H - 1, y + hi)
            x0, x1 = max(0, x + lo), min(W - 1, x + hi)
            out[y, x] = m[y0:y1 + 1, x0:x1 + 1].any()
    return out


def tile_flags(dilated: np.ndarray, tile_w: int, tile_h: int) -> np.ndarray:
    """bool [grid_h * grid_w] (row-major tile index): the tile holds a set dilated pixel."""
    d = np.asarray(dilated, bool)
    H, W = d.shape
    gw, gh = -(-W // tile_w), -(-H // tile_h)
    out = np.zeros(gh * gw, bool)
    for ty in range(gh):
        for tx in range(gw):
            out[ty * gw + tx] = d[ty * tile_h:(ty + 1) * tile_h, tx * tile_w:(tx + 1) * tile_w].any()
    return out


def masked_l1(render, gt, pixel_mask):
    """render, gt [C][H][W]; pixel_mask [H][W] -> (loss, grad): sum over masked pixels of |r - g| / (C H W),
    grad sign(r - g) / (C H W) on masked pixels and 0 elsewhere."""
    r = np.asarray(render, np.float64)
    g = np.asarray(gt, np.float64)
    m = np.broadcast_to(np.asarray(pixel_mask, bool)[None], r.shape)
    diff = r - g
    loss = float(np.abs(diff)[m].sum() / diff.size)
    grad = np.where(m, np.sign(diff) / diff.size, 0.0)
    return loss, grad


def masked_iterations(total: int, fraction: float) -> int:
    """Number of masked iterations at the start of a frame's fit."""
    return int(math.ceil(fraction * total - 1e-12))
