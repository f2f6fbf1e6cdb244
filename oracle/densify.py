"""Per-frame densification (the 3D-GS densification stage the paper applies at every time step), FP64 numpy
(oracle; test only).

The paper runs 3D-GS's densification inside each frame's fit (Sec. 3.4, last paragraph; implementation
details: from epoch 6 until 80% of the epochs, every 2 epochs, gradient threshold 0.00125 on N3DV).  What the
stage does is 3D-GS's, read here as:
    * statistic: per Gaussian, the running sum over iterations of the norm of the viewspace gradient in
      normalised device coordinates, |(W/2 dL/dx', H/2 dL/dy')|, and the number of iterations in which the
      Gaussian was visible (a non-empty tile rectangle); the score is their ratio (0 if never visible);
    * a Gaussian with score >= threshold is cloned when its largest scale is at most percent_dense x extent
      (0.01 x the camera extent), and split otherwise; after the stage every statistic restarts at zero;
    * pruning: a Gaussian whose opacity is below 0.005 is removed (3D-GS prunes in the same stage);
    * the new set keeps each Gaussian's children in place, in the order of their parents: a kept Gaussian has
      one child (itself), a clone two (itself, then its copy), a split two, a pruned one none;
    * split children: scale divided by 1.6 (log-scale - ln 1.6) and position p + R(q) (s * z) with z a standard
      normal 3-vector per child, R and s those of the parent; every other attribute is copied;
    * clone children: two coincident copies of opacity o' = 1 - sqrt(1 - o) (the rule of Kheradmand et al.,
      "3D Gaussian Splatting as Markov Chain Monte Carlo", for N copies 1 - (1 - o)^(1/N)), so that the pair
      composites like the parent where its Gaussian factor is 1 (1 - (1 - o')^2 = o); the plain 3D-GS clone
      copies o unchanged, which doubles the clone's weight and, with residuals that move in quantised steps,
      leaves it there;
    * QUEEN's residual parameters (latents, pre-gate position residual, gate logit) are copied to every child,
      so a child decodes like its parent; the split's offset and scale change are applied to the stored
      A_{t-1} of the children, so the decoded child is the split of the decoded parent;
    * Adam moments restart at zero for new Gaussians (a clone's copy and both split children); a clone's first
      child and a kept Gaussian keep theirs.
Pinned by: clones are exact copies apart from the opacity, and two coincident clones composite like their parent
at its centre; a split with z = 0 keeps the parent's mean; the children's mean offset is
R(q) (s * z) (rotation of a scaled vector, checked against an explicit rotation matrix built from the
quaternion's closed form); counts n' = n - pruned + clones + splits; the rank of the schedule's densification
iterations.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox

KEEP, CLONE, SPLIT, PRUNE = 0, 1, 2, 3
SPLIT_SCALE = 1.6
MIN_OPACITY = 0.005
PERCENT_DENSE = 0.01


def accumulate(accum, count, grad_xy, ntiles, sx, sy):
    """One iteration's statistic: grad_xy [2, n] (dL/dp' of one view, pixels), ntiles [n] of that view."""
    g = np.asarray(grad_xy, np.float64)
    vis = np.asarray(ntiles) > 0
    nrm = np.hypot(sx * g[0], sy * g[1])
    return accum + np.where(vis, nrm, 0.0), count + vis.astype(np.float64)


def plan(accum, count, log_scales, logits, threshold, max_scale, min_opacity=MIN_OPACITY):
    """Action per Gaussian (KEEP, CLONE, SPLIT, PRUNE) from the statistic and the decoded attributes
    (log_scales [3, n], opacity logits [n]); pruning takes precedence."""
    accum = np.asarray(accum, np.float64)
    count = np.asarray(count, np.float64)
    score = np.where(count > 0, accum / np.where(count > 0, count, 1.0), 0.0)
    big = np.exp(np.asarray(log_scales, np.float64).max(0)) > max_scale
    act = np.full(len(accum), KEEP, np.int64)
    grow = score >= threshold
    act[grow & ~big] = CLONE
    act[grow & big] = SPLIT
    opac = 1.0 / (1.0 + np.exp(-np.asarray(logits, np.float64)))
    act[opac < min_opacity] = PRUNE
    return act


def children(act):
    return np.where(act == PRUNE, 0, np.where(act == KEEP, 1, 2))


def clone_logit(x):
    """Logit of o' = 1 - sqrt(1 - o) for o = sigmoid(x): log(1 - s) - log(s) with s = sqrt(sigmoid(-x))."""
    s = math.sqrt(1.0 / (1.0 + math.exp(x)))
    return math.log1p(-s) - math.log(s)


def quat_matrix(q):
    """Rotation matrices [n, 3, 3] of the normalised quaternions q [n, 4] (w, x, y, z), closed form."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)


def apply(act, prev, decoded, params, moments, seed, rnd, normals=None):
    """The new arrays after the stage.

    act [n]; prev [59, n] (A_{t-1}); decoded [59, n] (the current decoded attributes: R and s of a split);
    params: list of [k, n] arrays copied to every child (latents, l_p, a ...); moments: list of [k, n] arrays
    (Adam m, v) that restart at zero for new Gaussians.  normals [n, 6] (optional) replaces the generator's
    split normals.  Returns (new prev [59, n'], new params, new moments, parent index [n'])."""
    act = np.asarray(act)
    n = len(act)
    k = children(act)
    parent = np.repeat(np.arange(n), k)
    first = np.concatenate([[True], parent[1:] != parent[:-1]]) if len(parent) else np.zeros(0, bool)
    new_prev = np.asarray(prev, np.float64)[:, parent].copy()
    new_params = [np.asarray(p)[:, parent].copy() for p in params]
    keepm = ((act[parent] == KEEP) | (act[parent] == CLONE)) & first
    new_moments = [np.where(keepm[None, :], np.asarray(m)[:, parent], 0.0) for m in moments]
    # clone children: stored logit moved so that the decoded opacity becomes o' = 1 - sqrt(1 - o)
    for out_j in np.flatnonzero(act[parent] == CLONE):
        i = int(parent[out_j])
        x = float(np.asarray(decoded, np.float64)[10, i])
        new_prev[10, out_j] += clone_logit(x) - x
    split_idx = np.flatnonzero(act == SPLIT)
    if len(split_idx):
        z = philox.split_normals(split_idx, seed, rnd) if normals is None else np.asarray(normals)[split_idx]
        R = quat_matrix(np.asarray(decoded, np.float64)[3:7, split_idx].T)
        s = np.exp(np.asarray(decoded, np.float64)[7:10, split_idx].T)
        pos = {int(i): j for j, i in enumerate(split_idx)}
        for out_j in np.flatnonzero(act[parent] == SPLIT):
            i = int(parent[out_j])
            j = pos[i]
            zz = z[j, 0:3] if first[out_j] else z[j, 3:6]
            new_prev[0:3, out_j] += R[j] @ (s[j] * zz)
            new_prev[7:10, out_j] -= math.log(SPLIT_SCALE)
    return new_prev, new_params, new_moments, parent


def schedule(iters_per_epoch, epochs, start_epoch=6, stop_frac=0.8, every=2):
    """Iterations (0-based, counted before the step runs) at which the stage runs: the start of epochs
    start_epoch, start_epoch + every, ... up to stop_frac of the epochs."""
    last = int(math.floor(stop_frac * epochs))
    return [e * iters_per_epoch for e in range(start_epoch, last + 1, every)]


def camera_extent(centres):
    """3D-GS's scene extent: 1.1 x the largest distance of a camera centre from their mean."""
    c = np.asarray(centres, np.float64)
    return 1.1 * float(np.linalg.norm(c - c.mean(0), axis=1).max())
