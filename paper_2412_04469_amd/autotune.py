"""Blend-schedule autotuner for the batched fit step.

The tile shape (8x8, 16x16, 32x8), the LDS batch depth of the blend kernels (32, 64, 128 entries) and the
work distribution (one workgroup per tile, or a resident grid taking tiles heaviest-first) change how the
blend and its adjoint run, never what they compute: images, T_final and last are bit-identical across
all of them, and the adjoint differs only in the order of its float atomics.  The autotuner therefore
times the real captured step of each candidate on the real inputs and keeps the fastest.
"""
from __future__ import annotations

import itertools
import time

import torch

TILES = ((16, 16), (8, 8), (32, 8))
BATCHES = (32, 64, 128)
PERSISTENT = (False, True)


def candidates(tiles=TILES, batches=BATCHES, persistent=PERSISTENT):
    return [dict(tile=t, batch=b, persistent=p) for t, b, p in itertools.product(tiles, batches, persistent)]


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


def autotune(make_fitter, cands=None, steps: int = 6, warmup: int = 2, log=None):
    """make_fitter(tile=..., batch=..., persistent=...) -> a sized BatchedFitter on the workload to tune.

    Each candidate is built, stepped `warmup` times (the first step of each view group is eager and captures
    the group's graph) and timed over `steps` graph replays.  Returns (best candidate, [(candidate, ms)]).
    Candidates that overflow their pair capacity are re-sized once and timed again."""
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
    return best, table
