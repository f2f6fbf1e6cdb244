"""Streaming reconstruction over a dynamic sequence, and the learned residual proposal judged against zero
initialisation.

Frame 0 is the true scene (it stands in for the first-frame training).  Each later frame t fits the
residuals of A_t = A_{t-1} + R_t (Eq. 4) on the 20 training views: Eq. 9-10 gate initialisation, then
optimiser iterations; the held-out centre view is scored every `check_every` iterations with the frame
clock paused.  The plain run records, per frame, the held-out PSNR after its full iteration budget (the
frame's target), the clock time at which it first reached that PSNR, the reconstruction A_t, the decoder
at the start of the frame, the fitted residual parameters (l_p, a, latents) and the Eq. 10 probabilities.

The proposal is trained on frames 1..25 of that record (features from A_{t-1}, A_{t-2}, A_{t-3} and the
Eq. 10 probabilities; targets the fitted parameters) and judged on frames 26..50: each judged frame starts
from the plain run's A_{t-1} and decoder, so both forms chase the same target from the same state; the
frame clock covers gate initialisation, features, the network and the fitting until the held-out PSNR
first reaches the target.  If the proposal's initial training loss is worse than that of zero-initialised
residuals, the frame falls back to zero initialisation (counted).
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import qg, synth
from .fit import BatchedFitter, FitConfig, FrameFitter, GateInitializer, render_views
from .proposal import Proposal, features


def _planes(scene, dev):
    return torch.as_tensor(scene.planes()).to(dev)


class Sequence:
    """Ground truth of the dynamic workload, rendered on demand (deterministic)."""

    def __init__(self, wl, cfg: FitConfig, dev):
        self.wl, self.cfg, self.dev = wl, cfg, dev
        self.motion = wl.extras["motion"]
        self.held = wl.extras["held_out"]

    def truth(self, t):
        return _planes(synth.frame_scene(self.wl.scene, self.motion, t), self.dev)

    def gts(self, t):
        tr = self.truth(t)
        views = render_views(tr, self.wl.cams, self.cfg)
        held = render_views(tr, [self.held], self.cfg)[0]
        return views, held


def _check_capacity(fitter):
    r = fitter.rast if hasattr(fitter, "rast") else None
    if r is not None and r.overflowed():
        r._alloc_capacity(int(r.pair_count() * 1.3))
        return True
    if hasattr(fitter, "rasts") and fitter.overflowed():
        fitter.size_capacity()
        return True
    return False


def fit_frame(fitter, step_fn, iters, check_every, held, gt_held, target=None, t_start=None):
    """Runs optimiser steps with a held-out check every check_every steps (clock paused during checks).
    Returns (trajectory [(iteration, seconds, psnr)], seconds at the first check >= target or None, overflows).
    The clock starts at t_start (perf_counter value; the caller's set-up work before it counts)."""
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    traj, hit, ovf = [], None, 0
    it = 0
    while it < iters:
        t0 = time.perf_counter()
        for _ in range(min(check_every, iters - it)):
            step_fn(it)
            it += 1
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        ovf += int(_check_capacity(fitter))
        p = fitter.psnr(held, gt_held)
        traj.append((it, round(elapsed, 4), round(p, 3)))
        if target is not None and p >= target:
            hit = elapsed
            break
    return traj, hit, ovf


def fitted_params(f):
    """[12][n] = [l_p (3) | a (1) | latents (8)] of a fitter."""
    return torch.cat([f.lp, f.a[None], f.lat], 0)


def run_plain(seq: Sequence, frames, iters=500, check_every=25, log=None, capacity_margin=1.3):
    """Plain streaming fit over frames 1..frames.  Returns (per-frame records, history dict)."""
    cfg, dev, wl = seq.cfg, seq.dev, seq.wl
    A = seq.truth(0)
    gts_prev, _ = seq.gts(0)
    fitter = FrameFitter(A, wl.cams, gts_prev, cfg)
    fitter.size_capacity(capacity_margin)
    gi = GateInitializer(fitter.n, wl.cams, cfg)
    gi(A, gts_prev, gts_prev)  # buffers warm
    order = np.random.default_rng(0)
    V = len(wl.cams)
    hist = {"A": {0: A.clone()}, "W": {}, "y": {}, "p": {}}
    recs = []
    for t in range(1, frames + 1):
        gts, gt_held = seq.gts(t)
        hist["W"][t] = (fitter.W1.clone(), fitter.W2.clone())
        perm = np.concatenate([order.permutation(V) for _ in range(iters // V + 2)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a0 = gi(A, gts_prev, gts)
        fitter.reset_frame(prev_attrs=A, gts=gts, a_init=a0)
        traj, _, ovf = fit_frame(fitter, lambda i: fitter.step(int(perm[i])), iters, check_every, seq.held, gt_held,
                                 t_start=t0)
        target = traj[-1][2]
        hit = next(s for (i, s, p) in traj if p >= target)
        fitter.decode()
        A = fitter.attrs.clone()
        hist["A"][t] = A
        hist["y"][t] = fitted_params(fitter).clone()
        hist["p"][t] = gi.p.clone()
        recs.append(dict(t=t, target=target, sec=round(hit, 4), iters_to_target=next(i for (i, s, p) in traj
                                                                                       if p >= target),
                         psnr_first=traj[0][2], overflows=ovf))
        if log:
            log(f"plain frame {t}: {target:.3f} dB, {hit:.3f} s")
        gts_prev = gts
    return recs, hist


def proposal_inputs(hist, t, p):
    A = hist["A"]
    a1, a2, a3 = A[t - 1], A[max(t - 2, 0)], A[max(t - 3, 0)]
    return features(a1, a2, a3, p)


def train_proposal(hist, frames, steps=800, batch=65536, lr=2e-3, seed=0, log=None):
    X = torch.cat([proposal_inputs(hist, t, hist["p"][t]) for t in frames], 1).contiguous()
    Y = torch.cat([hist["y"][t] for t in frames], 1).contiguous()
    prop = Proposal(seed=seed, lr=lr)
    prop.set_stats(X, Y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = prop.train(X, Y, steps=steps, batch=batch, log_every=max(steps // 8, 1), log=log)
    torch.cuda.synchronize()
    return prop, losses, time.perf_counter() - t0


def _train_loss(fitter, views):
    """Mean L1 over some training views at the current parameters (host sync)."""
    tot = 0.0
    fitter.decode()
    for v in views:
        fitter.forward_view(v)
        qg.qg_l1_loss(fitter.count, fitter.rast.images[0], fitter.gts[v], 1.0, None, fitter.loss_part)
        qg.qg_loss_reduce(fitter.count, fitter.loss_part, fitter.loss_out)
        tot += float(fitter.loss_out[0].item())
    fitter.loss_tiles = 0  # its partials now hold these blocks, not a step's per-tile sums
    return tot / len(views)


def judge(seq: Sequence, hist, plain_recs, prop: Proposal, frames, iters=500, check_every=25, batched=False,
          log=None, capacity_margin=1.3, budget=2.0, batched_cfg=None):
    """Proposal-initialised fitting on the given frames, from the plain run's A_{t-1} and decoder; each frame
    may run up to budget x iters steps to reach the plain form's target.  batched_cfg: the FitConfig of the
    batched fitter (views per step, learning-rate scale), the sequence's by default."""
    cfg, dev, wl = seq.cfg, seq.dev, seq.wl
    targets = {r["t"]: r["target"] for r in plain_recs}
    A0 = hist["A"][frames[0] - 1]
    gts0, _ = seq.gts(frames[0] - 1)
    if batched:
        fitter = BatchedFitter(A0, wl.cams, gts0, batched_cfg or cfg, eval_cam=seq.held)
        fitter.size_capacity(capacity_margin)
        probe = FrameFitter(A0, wl.cams, gts0, cfg)  # single-view renders for the fallback check
        probe.size_capacity(capacity_margin)
    else:
        fitter = FrameFitter(A0, wl.cams, gts0, cfg)
        fitter.size_capacity(capacity_margin)
        probe = fitter
    if batched:
        for _ in fitter.groups:  # capture every group's step before any frame clock runs
            fitter.step()
    gi = GateInitializer(fitter.n, wl.cams, cfg)
    order = np.random.default_rng(1)
    V = len(wl.cams)
    recs = []
    for t in frames:
        A = hist["A"][t - 1]
        gts_prev, _ = seq.gts(t - 1)
        gts, gt_held = seq.gts(t)
        W1, W2 = hist["W"][t]
        fitter.W1.copy_(W1)
        fitter.W2.copy_(W2)
        if probe is not fitter:
            probe.W1.copy_(W1)
            probe.W2.copy_(W2)
        perm = np.concatenate([order.permutation(V) for _ in range(int(budget * iters) // V + 2)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a_eq10 = gi(A, gts_prev, gts).clone()
        y = prop.predict(proposal_inputs(hist, t, gi.p))
        # fallback check on two training views: proposal initialisation against zero initialisation
        check_views = [0, V // 2]
        probe.reset_frame(prev_attrs=A, gts=gts, a_init=a_eq10)
        zero_loss = _train_loss(probe, check_views)
        probe.reset_frame(prev_attrs=A, gts=gts, a_init=y[3], lat_init=y[4:12], lp_init=y[0:3])
        prop_loss = _train_loss(probe, check_views)
        use_prop = prop_loss <= zero_loss
        if use_prop:
            fitter.reset_frame(prev_attrs=A, gts=gts, a_init=y[3], lat_init=y[4:12], lp_init=y[0:3])
        else:
            fitter.reset_frame(prev_attrs=A, gts=gts, a_init=a_eq10)
        if batched:
            step = lambda i: fitter.step()
        else:
            step = lambda i: fitter.step(int(perm[i]))
        traj, hit, ovf = fit_frame(fitter, step, int(budget * iters), check_every, seq.held, gt_held,
                                   target=targets[t], t_start=t0)
        recs.append(dict(t=t, target=targets[t], sec=None if hit is None else round(hit, 4), used_proposal=use_prop,
                         init_loss=(round(zero_loss, 6), round(prop_loss, 6)), psnr_first=traj[0][2],
                         iters_to_target=traj[-1][0] if hit is not None else None, overflows=ovf))
        if log:
            log(f"{'batched ' if batched else ''}proposal frame {t}: "
                f"{'%.3f s' % hit if hit is not None else 'target not reached'} (proposal used: {use_prop})")
    return recs


def summarize(plain_recs, judged, frames):
    plain = [r for r in plain_recs if r["t"] in frames]
    ps = [r["sec"] for r in plain]
    js = [r["sec"] for r in judged]
    reached = [s for s in js if s is not None]
    return {"frames": [min(frames), max(frames)],
            "plain_mean_sec_per_frame": round(float(np.mean(ps)), 4),
            "mean_sec_per_frame": round(float(np.mean(reached)), 4) if len(reached) == len(js) else None,
            "mean_sec_per_frame_reached": round(float(np.mean(reached)), 4) if reached else None,
            "frames_reaching_target": len(reached), "frames_using_proposal": sum(r["used_proposal"] for r in judged),
            "mean_iters_to_target": round(float(np.mean([r["iters_to_target"] for r in judged
                                                          if r["iters_to_target"] is not None])), 1)
            if reached else None,
            "plain_mean_iters_to_target": round(float(np.mean([r["iters_to_target"] for r in plain])), 1)}
