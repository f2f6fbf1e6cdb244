"""Independent NumPy compositor for tiny scenes (oracle; test only).

Written separately from ``composite.c`` from the same definition (Eq. 2 with the 1/255 skip, the 0.99
clamp and termination before T' < 1e-4) so that each pins the other.  Pure-Python loop over pixels and
contributors; use only for a few hundred splats and at most 64x64 pixels.
"""
from __future__ import annotations

import numpy as np


def render(xy, conic, opacity, rgb, depth, width, height, bg=(0.0, 0.0, 0.0), valid=None,
           alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4):
    xy = np.asarray(xy, np.float64)
    A, B, C = (np.asarray(conic, np.float64)[:, k] for k in range(3))
    o = np.asarray(opacity, np.float64)
    col = np.asarray(rgb, np.float64)
    dep = np.asarray(depth, np.float64)
    n = len(o)
    keep = np.ones(n, bool) if valid is None else np.asarray(valid, bool)
    order = np.lexsort((np.arange(n), dep))  # by depth, then index
    order = order[keep[order]]
    img = np.zeros((3, height, width))
    tf = np.zeros((height, width))
    last = np.full((height, width), -1, np.int64)
    for i in range(height):
        for j in range(width):
            dx = j + 0.5 - xy[order, 0]
            dy = i + 0.5 - xy[order, 1]
            a = o[order] * np.exp(-0.5 * (A[order] * dx * dx + 2 * B[order] * dx * dy + C[order] * dy * dy))
            a = np.minimum(a, alpha_max)
            T = 1.0
            acc = np.zeros(3)
            for kk in np.flatnonzero(a >= alpha_min):
                nt = T * (1.0 - a[kk])
                if nt < t_min:
                    break
                acc += col[order[kk]] * a[kk] * T
                T = nt
                last[i, j] = order[kk]
            img[:, i, j] = acc + T * np.asarray(bg, np.float64)
            tf[i, j] = T
    return img, tf, last
