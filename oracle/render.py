"""The oracle's whole chain: planes -> projection (torch FP64) -> per-pixel compositing (C FP64) and back.

Test infrastructure only.  The backward runs the C adjoint of Eq. 2 for the 2D splat quantities and then
torch autograd through the projection/decode formulas, so no hand-derived chain rule is shared with the
kernels under test.
"""
from __future__ import annotations

import numpy as np
import torch

from . import composite as _comp
from . import project as _proj


def unpack(planes: torch.Tensor):
    n = planes.shape[1]
    return (planes[0:3].T, planes[3:7].T, planes[7:10].T, planes[10], planes[11:59].T.reshape(n, 16, 3))


def splats_numpy(pr: dict) -> dict:
    return {"xy": pr["xy"].detach().numpy(), "conic": pr["conic"].detach().numpy(),
            "opacity": pr["opacity"].detach().numpy(), "rgb": pr["rgb"].detach().numpy(),
            "depth": pr["depth"].detach().numpy(), "valid": pr["valid"].numpy()}


def render(planes, cam, bg=(0.0, 0.0, 0.0), sh_degree=3, dilation=_proj.DILATION, grad_image=None,
           pixels=None, **kw):
    """Render one camera.

    planes: float64 torch tensor [59,N] (set ``requires_grad`` to get ``planes.grad``) or a numpy array.
    pixels: optional (px, py) centre coordinates; otherwise the whole image.
    grad_image: dL/dimage, [3,H,W] for the whole image or [M,3] for a pixel list.
    Returns dict with the projection, the composite outputs and (if grad_image) the 2D gradients.
    """
    if not isinstance(planes, torch.Tensor):
        planes = torch.tensor(np.asarray(planes, np.float64))
    means, quats, ls, logits, sh = unpack(planes)
    pr = _proj.project(means, quats, ls, logits, sh, cam, sh_degree, dilation)
    sp = splats_numpy(pr)
    if pixels is None:
        out = _comp.composite_image(sp, cam.width, cam.height, bg, grad_image, **kw)
    else:
        out = _comp.composite(sp, pixels[0], pixels[1], bg, grad_image, **kw)
    out["proj"] = pr
    out["splats"] = sp
    if grad_image is not None and planes.requires_grad:
        ts = [pr["xy"], pr["conic"], pr["opacity"], pr["rgb"]]
        gs = [torch.tensor(out[k]) for k in ("g_xy", "g_conic", "g_opacity", "g_rgb")]
        torch.autograd.backward(ts, gs)
    return out
