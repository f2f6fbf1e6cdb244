"""Shared test helpers: build inputs from the generator, run the HIP path through the C ABI, run the oracle."""
from __future__ import annotations

import numpy as np
import torch

from paper_2412_04469_amd import synth

MARGIN_FWD = 1e-4   # relative alpha/termination margin below which float32 may decide differently
MARGIN_ORDER = 1e-6  # relative depth gap below which independently computed float32 depths may swap


def keep_mask(ref, order=True, margin=MARGIN_FWD):
    """Pixels whose oracle decisions are far enough from their thresholds to be compared; prints how many are
    left out."""
    k = ref["margin"] >= margin
    if order:
        k &= ref["order_margin"] >= MARGIN_ORDER
    print(f"[margins] {int(k.size - k.sum())} of {k.size} pixels excluded", flush=True)
    return k


def small_scene(seed=10, n=3000, mean_std=1.0, ls_mu=-3.5, ls_std=0.5):
    return synth.draw_scene(synth.rng_for(seed), n, mean_std, ls_mu, ls_std)


def cams_small(width=160, height=120):
    return [synth.make_camera((0.0, 0.0, -4.0), width, height, f=width),
            synth.make_camera((1.5, -0.6, -3.5), width, height, f=width * 0.9)]


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def splat_fields(proj_bufs):
    """Host numpy views of a projected buffer dict (one view)."""
    sp = proj_bufs["splat"].cpu().numpy()
    return {"xy": sp[:, 0:2], "opacity": sp[:, 2], "conic": sp[:, 4:7], "rgb": sp[:, 8:11],
            "depth": proj_bufs["depth"].cpu().numpy(), "rect": proj_bufs["rect"].cpu().numpy(),
            "ntiles": proj_bufs["ntiles"].cpu().numpy(), "flags": proj_bufs["flags"].cpu().numpy()}


def rel_l2(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))
