"""Tile binning by (tile, depth) keys and a stable sort, written as the plain definition (oracle; test only).

The paper only states that the N Gaussians are blended in depth order (Sec. 3.1, Eq. 2).  The tiled
form orders, for every tile, the Gaussians whose tile rectangle covers it by (depth, index):
    key = (global tile id << 32) | float32 bit pattern of the depth (positive, so monotone as unsigned)
    value = Gaussian index
Pairs are enumerated Gaussian by Gaussian (index order) and tile by tile (row-major inside the
rectangle); a stable sort of the keys then breaks equal keys by index.  Tile ranges give, for each tile,
the half-open span of its pairs in the sorted array ([0, 0) for an empty tile).

Pinned by brute force: for every tile, the list of Gaussians whose rectangle covers it, ordered by
(depth bits, index) directly, must equal the tile's span of the sorted values.
"""
from __future__ import annotations

import numpy as np


def make_pairs(rect: np.ndarray, depth_f32: np.ndarray, grid_w: int, tile_offset: int = 0):
    """Enumerate (key, value) pairs.  rect [N,4] half-open (tx0, ty0, tx1, ty1); depth_f32 float32 [N]."""
    rect = np.asarray(rect, np.int64)
    bits = np.asarray(depth_f32, np.float32).view(np.uint32).astype(np.uint64)
    keys, vals = [], []
    for i in range(rect.shape[0]):
        tx0, ty0, tx1, ty1 = rect[i]
        for ty in range(ty0, ty1):
            for tx in range(tx0, tx1):
                tile = tile_offset + ty * grid_w + tx
                keys.append((np.uint64(tile) << np.uint64(32)) | bits[i])
                vals.append(i)
    return np.array(keys, np.uint64), np.array(vals, np.uint32)


def make_pairs_fast(rect: np.ndarray, depth_f32: np.ndarray, grid_w: int, tile_offset: int = 0):
    """Vectorised enumeration in the same order as ``make_pairs``."""
    rect = np.asarray(rect, np.int64)
    w = np.maximum(rect[:, 2] - rect[:, 0], 0)
    h = np.maximum(rect[:, 3] - rect[:, 1], 0)
    cnt = w * h
    total = int(cnt.sum())
    idx = np.repeat(np.arange(rect.shape[0], dtype=np.int64), cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(total, dtype=np.int64) - start
    wi = np.maximum(w[idx], 1)
    ty = rect[idx, 1] + local // wi
    tx = rect[idx, 0] + local % wi
    tile = (tile_offset + ty * grid_w + tx).astype(np.uint64)
    bits = np.asarray(depth_f32, np.float32).view(np.uint32).astype(np.uint64)
    keys = (tile << np.uint64(32)) | bits[idx]
    return keys, idx.astype(np.uint32)


def sort_pairs(keys: np.ndarray, vals: np.ndarray):
    order = np.argsort(keys, kind="stable")
    return keys[order], vals[order]


def tile_ranges(sorted_keys: np.ndarray, n_tiles: int) -> np.ndarray:
    """[n_tiles, 2] uint32 half-open spans; empty tiles get [0, 0)."""
    out = np.zeros((n_tiles, 2), np.uint32)
    if sorted_keys.size == 0:
        return out
    tiles = (sorted_keys >> np.uint64(32)).astype(np.int64)
    starts = np.flatnonzero(np.r_[True, tiles[1:] != tiles[:-1]])
    ends = np.r_[starts[1:], tiles.size]
    out[tiles[starts], 0] = starts
    out[tiles[starts], 1] = ends
    return out


def bin_view(rect, depth_f32, grid_w, grid_h, tile_offset=0):
    keys, vals = make_pairs_fast(rect, depth_f32, grid_w, tile_offset)
    k, v = sort_pairs(keys, vals)
    return k, v, tile_ranges(k, tile_offset + grid_w * grid_h)
