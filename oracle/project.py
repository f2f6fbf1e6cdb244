"""Covariance, EWA projection (Eq. 1), SH colour and splat support, in torch FP64 (oracle; test only).

Definitions (paper Sec. 3.1, "Representation" and "Rendering"):
    Sigma = R(q) S S^T R(q)^T, S = diag(s)                          (quaternion q, scale s)
    p' = Pi(p; K, W),  Sigma' = J W Sigma W^T J^T                     (Eq. 1; J = Jacobian of the affine
                                                                      approximation of the projection)
Readings where the paper is silent (listed in the design notes):
    * q is stored unnormalised in (w, x, y, z) order and normalised before use; s = exp(log-scale);
      opacity o = sigmoid(logit).
    * camera: OpenCV axes, world->camera u = R p + t, p' = (fx ux/uz + cx, fy uy/uz + cy); pixel (i, j)
      has its centre at (j + 0.5, i + 0.5).  A Gaussian is culled if uz <= z_near, if Sigma' is not
      positive definite, if any input is non-finite or if o < 1/255 (it can never reach alpha >= 1/255).
    * J = [[fx/uz, 0, -fx ux/uz^2], [0, fy/uz, -fy uy/uz^2]] with no frustum clamp.
    * a low-pass dilation h (0.3 px^2 by default) is added to the diagonal of Sigma'.
    * conic = Sigma'^{-1} stored as (A, B, C) in q = A dx^2 + 2 B dx dy + C dy^2.
    * colour c = max(0, sum_k h_k Y_k(dir) + 0.5), dir = (p - c_cam)/|p - c_cam|, c_cam = -R^T t.
    * depth used for ordering = uz (camera-space z).
    * support: alpha >= 1/255 <=> dx^T conic d <= k^2 = 2 ln(255 o); the axis-aligned half extents of that
      ellipse are k sqrt(Sigma'_xx) and k sqrt(Sigma'_yy); covered pixels are those whose centres lie in
      [p' - r, p' + r]; the tile rectangle is the set of tiles holding a covered pixel, clipped to the image.

Pinned by closed forms (on-axis and off-axis Sigma'), Monte-Carlo convergence of the projected sample
covariance, rigid-motion invariance, SH quadrature, textbook degree-1..3 SH values along the direction from a
rotated, translated camera's centre to the mean (a reversed direction flips the odd degrees), and for the
rectangle: a brute-force check that every pixel with alpha >= 1/255 lies in a tile of the rectangle
(containment), the exact rectangles of an isotropic splat whose support disc is known in closed form (one at
the image border), and a parametric sampling of the support ellipse's extent (tightness).  Gradients come from torch autograd
applied to these plain formulas.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import sh as _sh

DILATION = 0.3


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of a unit quaternion (w, x, y, z) [N,4] -> [N,3,3]."""
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def covariance(quats: torch.Tensor, log_scales: torch.Tensor) -> torch.Tensor:
    q = quats / torch.linalg.vector_norm(quats, dim=-1, keepdim=True)
    Rq = quat_to_rot(q)
    M = Rq * torch.exp(log_scales)[:, None, :]  # M = R S
    return M @ M.transpose(1, 2)


def cam_tensors(cam):
    R = torch.as_tensor(np.asarray(cam.R, np.float64))
    t = torch.as_tensor(np.asarray(cam.t, np.float64))
    return R, t


def project(means, quats, log_scales, logits, sh, cam, sh_degree: int = 3, dilation: float = DILATION):
    """Project N Gaussians (torch float64 tensors) into one camera.

    Returns a dict of tensors: xy [N,2], conic [N,3], cov2d [N,3] (a, b, c of Sigma'), depth [N], opacity [N],
    rgb [N,3], rgb_pre [N,3] and a bool ``valid`` [N].
    """
    R, t = cam_tensors(cam)
    u = means @ R.T + t
    ux, uy, uz = u.unbind(-1)
    finite = torch.isfinite(means).all(-1) & torch.isfinite(quats).all(-1) & torch.isfinite(log_scales).all(-1) \
        & torch.isfinite(logits) & torch.isfinite(sh.reshape(sh.shape[0], -1)).all(-1)
    front = uz > cam.z_near
    ok = finite & front
    one = torch.ones_like(uz)
    uzs = torch.where(ok, uz, one)
    uxs = torch.where(ok, ux, torch.zeros_like(ux))
    uys = torch.where(ok, uy, torch.zeros_like(uy))
    fx, fy = float(cam.fx), float(cam.fy)
    zero = torch.zeros_like(uzs)
    J = torch.stack([
        torch.stack([fx / uzs, zero, -fx * uxs / (uzs * uzs)], -1),
        torch.stack([zero, fy / uzs, -fy * uys / (uzs * uzs)], -1),
    ], -2)
    Tm = J @ R
    qs = torch.where(ok[:, None], quats, torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=quats.dtype))
    ls = torch.where(ok[:, None], log_scales, torch.zeros_like(log_scales))
    Sigma = covariance(qs, ls)
    cov = Tm @ Sigma @ Tm.transpose(1, 2)
    a = cov[:, 0, 0] + dilation
    b = cov[:, 0, 1]
    c = cov[:, 1, 1] + dilation
    det = a * c - b * b
    pd = ok & (det > 0) & (a > 0)
    dets = torch.where(pd, det, one)
    conic = torch.stack([c / dets, -b / dets, a / dets], -1)
    xy = torch.stack([fx * uxs / uzs + float(cam.cx), fy * uys / uzs + float(cam.cy)], -1)
    opacity = torch.sigmoid(logits)
    cc = -(R.T @ t)  # camera centre c_v = -R^T t (u = R p + t vanishes there)
    v = means - cc
    dirs = v / torch.linalg.vector_norm(v, dim=-1, keepdim=True)
    nb = (sh_degree + 1) ** 2
    Y = _sh.basis(torch.where(ok[:, None], dirs, torch.tensor([0.0, 0.0, 1.0], dtype=dirs.dtype)), sh_degree)
    rgb_pre = (Y[:, :, None] * sh[:, :nb, :]).sum(1) + 0.5
    rgb = torch.clamp_min(rgb_pre, 0.0)
    valid = pd & (opacity >= 1.0 / 255.0)
    return {"xy": xy, "conic": conic, "cov2d": torch.stack([a, b, c], -1), "depth": uz, "opacity": opacity,
            "rgb": rgb, "rgb_pre": rgb_pre, "valid": valid}


def pixel_rect(xy: np.ndarray, cov2d: np.ndarray, opacity: np.ndarray, valid: np.ndarray, width: int, height: int):
    """Inclusive pixel rectangle [j0, j1] x [i0, i1] of covered pixel centres, clipped to the image.

    Returns (j0, j1, i0, i1, empty, edges) where ``edges`` holds the real-valued bounds
    (x - rx - 0.5, x + rx - 0.5, y - ry - 0.5, y + ry - 0.5) before rounding."""
    xy = np.asarray(xy, np.float64)
    cov2d = np.asarray(cov2d, np.float64)
    o = np.asarray(opacity, np.float64)
    ok = np.asarray(valid, bool) & (255.0 * o >= 1.0)
    k2 = 2.0 * np.log(np.where(ok, 255.0 * o, 1.0))
    k = np.sqrt(k2)
    rx = k * np.sqrt(np.where(ok, cov2d[:, 0], 0.0))
    ry = k * np.sqrt(np.where(ok, cov2d[:, 2], 0.0))
    x = np.where(ok, xy[:, 0], -1e9)
    y = np.where(ok, xy[:, 1], -1e9)
    edges = np.stack([x - rx - 0.5, x + rx - 0.5, y - ry - 0.5, y + ry - 0.5], 1)
    j0 = np.maximum(np.ceil(edges[:, 0]), 0)
    j1 = np.minimum(np.floor(edges[:, 1]), width - 1)
    i0 = np.maximum(np.ceil(edges[:, 2]), 0)
    i1 = np.minimum(np.floor(edges[:, 3]), height - 1)
    empty = ~ok | (j0 > j1) | (i0 > i1)
    return j0, j1, i0, i1, empty, edges


def tile_rect(xy, cov2d, opacity, valid, width, height, tile_w, tile_h):
    """Half-open tile rectangle (tx0, ty0, tx1, ty1) int32 [N,4] and tile count [N] (0 if nothing covered).

    Also returns the four real-valued rectangle edges so tests can flag cases within rounding
    distance of an integer boundary."""
    j0, j1, i0, i1, empty, edges = pixel_rect(xy, cov2d, opacity, valid, width, height)
    rect = np.zeros((len(j0), 4), np.int64)
    rect[:, 0] = np.floor_divide(j0, tile_w)
    rect[:, 1] = np.floor_divide(i0, tile_h)
    rect[:, 2] = np.floor_divide(j1, tile_w) + 1
    rect[:, 3] = np.floor_divide(i1, tile_h) + 1
    rect[empty] = 0
    ntiles = (rect[:, 2] - rect[:, 0]) * (rect[:, 3] - rect[:, 1])
    return rect.astype(np.int32), ntiles.astype(np.int64), edges


def scene_tensors(scene, requires_grad: bool = False):
    """float64 torch tensors from a synth.Scene (means, quats, log_scales, logits, sh)."""
    ts = [torch.tensor(np.asarray(a, np.float64)) for a in (scene.means, scene.quats, scene.log_scales,
                                                               scene.logits, scene.sh)]
    if requires_grad:
        for t in ts:
            t.requires_grad_(True)
    return ts
