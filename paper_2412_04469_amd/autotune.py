"""Autotuning of the batched fit: the blend schedule of the step, and the step grouping of the frame.

Blend schedule.  The tile shape (8x8, 16x16, 32x8), the LDS batch depth of the blend kernels (32, 64, 128, 256
entries) and the tile order (groups of tiles dealt round-robin to the XCDs, or heaviest first) change how the
blend and its adjoint run, never what they compute: images, T_final and last are bit-identical
across all of them, and the adjoint differs only in the order of its float atomics.  The autotuner therefore
times the real captured step of each candidate on the real inputs and keeps the fastest.  Choices can be kept
in a JSON cache file, keyed by device, resolution bucket, Gaussian-count bucket and view count.

Step grouping.  How many views one optimiser step covers and the factor on the learning rates change the
optimisation itself, so they are chosen by what they are for: the seconds a frame's fit needs to reach the
plain form's target PSNR, measured on a tuning frame (not on the frames that are then judged).
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

import torch

TILES = ((16, 16), (8, 8), (32, 8))
BATCHES = (32, 64, 128, 256)
HEAVIEST_FIRST = (False, True)
# (views per step, learning-rate factor) candidates of the step grouping
GROUPINGS = ((2, 1.5), (4, 2.5), (5, 2.0), (10, 3.0))


def candidates(tiles=TILES, batches=BATCHES, heaviest_first=HEAVIEST_FIRST):
    return [dict(tile=t, batch=b, heaviest_first=h) for t, b, h in itertools.product(tiles, batches, heaviest_first)]


def time_steps(fitter, steps: int, warmup: int) -> float:
    """Mean ms per optimiser step over `steps` steps (after `warmup`), each group's graph replayed."""
    for _ in range(warmup):
        fitter.step()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fitter.step()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def cache_key(cams, n: int) -> str:
    """Device name, total pixels (power-of-two bucket in Mpx), Gaussian count (power-of-two bucket), views."""
    dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    px = sum(c.width * c.height for c in cams)
    return f"{dev}|px2^{round(math.log2(max(px, 1) / 1e6) if px else 0)}|n2^{round(math.log2(max(n, 1)))}|V{len(cams)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def autotune(make_fitter, cands=None, steps: int = 6, warmup: int = 2, log=None, cache_path=None, key=None):
    """make_fitter(tile=..., batch=..., heaviest_first=...) -> a sized BatchedFitter on the workload to tune.

    Each candidate is built, stepped `warmup` times (the first step of each view group is eager and captures
    the group's graph) and timed over `steps` graph replays.  Returns (best candidate, [(candidate, ms)]).
    Candidates that overflow their pair capacity are re-sized once and timed again.  With cache_path and key, a
    cached choice is returned without timing (table empty), and a new choice is stored."""
    if cache_path and key:
        hit = _load(cache_path).get(key)
        if hit:
            best = dict(tile=tuple(hit["tile"]), batch=int(hit["batch"]), heaviest_first=bool(hit["heaviest_first"]))
            if log:
                log(f"autotune: cached choice {best} for {key}")
            return best, []
    cands = candidates() if cands is None else cands
    table = []
    for c in cands:
        t0 = time.perf_counter()
        f = make_fitter(**c)
        ms = time_steps(f, steps, warmup + len(f.groups))
        if f.overflowed():
            f.size_capacity()
            ms = time_steps(f, steps, warmup + len(f.groups))
        table.append((c, ms))
        if log:
            log(f"autotune {c}: {ms:.3f} ms/step ({time.perf_counter() - t0:.1f} s)")
        del f
        torch.cuda.empty_cache()
    best = min(table, key=lambda cm: cm[1])[0]
    if cache_path and key:
        data = _load(cache_path)
        data[key] = dict(tile=list(best["tile"]), batch=best["batch"], heaviest_first=best["heaviest_first"],
                         ms=round(min(ms for _, ms in table), 4))
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return best, table


def tune_grouping(run_frame, groupings=GROUPINGS, log=None):
    """run_frame(views_per_step, lr_scale) -> seconds to the target PSNR on the tuning frame, or None if not
    reached.  Returns (best (views, lr) or None if no candidate reached the target, [(views, lr, seconds)])."""
    table = []
    for vps, lr in groupings:
        sec = run_frame(vps, lr)
        table.append((vps, lr, sec))
        if log:
            log(f"grouping {vps} views x lr {lr}: {'%.3f s' % sec if sec is not None else 'target not reached'}")
    reached = [(s, v, l) for v, l, s in table if s is not None]
    best = None if not reached else min(reached)[1:]
    return best, table
