"""Parity at the full workload sizes, on outputs the oracle can compute pixel by pixel (GPU).

* The per-frame fit workload (300 k Gaussians, 1352x1014) through the calls the benchmark step makes: fused
  decode+projection, binning, blend, fused adjoint.  Sampled pixels are compared with the FP64 oracle (image
  within 1e-4), and a sparse image gradient on the sampled pixels gives residual-parameter gradients that are
  compared with the oracle's (decode and projection through torch autograd, compositing in C) within 1e-3
  relative L2.
* The dense-overlap workload (1 M Gaussians, log-scales N(-3, 0.5), 4 views at 1920x1080, one multi-view call):
  sampled pixels and attribute gradients against the oracle, no capacity overflow.
* Its 2 k-Gaussian 64x64 sub-scene: whole-image attribute gradients against the oracle.
* The batched 12-view workload (500 k Gaussians at three resolutions) in one multi-view call per step: sampled
  pixels of three views and the residual-parameter gradients of a sparse image gradient over them.
Pixels whose oracle decision margin is below the usual thresholds are left out (and counted).
"""
import numpy as np
import pytest
import torch

from _helpers import MARGIN_FWD, MARGIN_ORDER, rel_l2, to_dev
from oracle import decode as OD
from oracle import render as OR
from paper_2412_04469_amd import synth

pytestmark = pytest.mark.gpu


def _candidates(rng, cam, m):
    idx = rng.choice(cam.width * cam.height, size=m, replace=False)
    return idx % cam.width, idx // cam.width


def _keep(ref):
    k = (ref["margin"] >= MARGIN_FWD) & (ref["order_margin"] >= MARGIN_ORDER)
    print(f"[margins] {int(k.size - k.sum())} of {k.size} pixels excluded", flush=True)
    return k


def _groups(g):
    return {"mean": g[0:3], "quat": g[3:7], "log_scale": g[7:10], "logit": g[10:11], "sh_dc": g[11:14],
            "sh_rest": g[14:59]}


def test_fit_workload_fullsize_sampled_parity():
    from paper_2412_04469_amd import qg
    from paper_2412_04469_amd.fit import FitConfig, FrameFitter
    wl = synth.workload_fit()
    n = wl.scene.n
    cfg = FitConfig()
    rng = np.random.default_rng(7)
    prev = wl.scene.planes()
    lat = rng.normal(0, 1.0, (8, n)).astype(np.float32)
    lp = rng.normal(0, 0.01, (3, n)).astype(np.float32)
    a = rng.normal(0, 1.0, n).astype(np.float32)
    cam = wl.cams[7]
    H, W = cam.height, cam.width
    f = FrameFitter(to_dev(prev), [cam], [torch.zeros(3, H, W, device="cuda")], cfg)
    f.lat.copy_(to_dev(lat))
    f.lp.copy_(to_dev(lp))
    f.a.copy_(to_dev(a))
    f.size_capacity()
    r = f.rast
    qg.qg_decode_project(n, f.ld, f.prev, f.lat, 8, f.W1, f.W2, 32, 56, f.lp, f.a, cfg.gamma0, cfg.gamma1, cfg.tau,
                         cfg.sh_degree, r.qcams, r.tile, cfg.dilation, r.t_proj, None, f.gate, None)
    r.bin()
    r.render()
    torch.cuda.synchronize()
    assert 0 < int(r.num_pairs.item()) <= r.capacity
    img = r.images[0].cpu().numpy()
    # oracle forward at candidate pixels (decode in FP64, straight-through rounding)
    hp = (cfg.gamma0, cfg.gamma1, cfg.tau)
    t = {k: torch.tensor(v.astype(np.float64), requires_grad=True)
         for k, v in (("lat", lat), ("W1", f.W1.cpu().numpy()), ("W2", f.W2.cpu().numpy()), ("lp", lp), ("a", a))}
    attrs, _, lreg = OD.decode(torch.tensor(prev.astype(np.float64)), t["lat"], t["W1"], t["W2"], t["lp"], t["a"], *hp)
    px, py = _candidates(rng, cam, 400)
    ref0 = OR.render(attrs.detach(), cam, cfg.bg, pixels=(px + 0.5, py + 0.5))
    keep = _keep(ref0)
    assert keep.mean() > 0.97, keep.mean()
    got = img[:, py, px].T
    assert np.abs(got - ref0["color"])[keep].max() <= 1e-4
    assert np.abs(r.tfinal[0].cpu().numpy()[py, px] - ref0["t_final"])[keep].max() <= 1e-4
    # sparse image gradient on 96 kept pixels
    sel = np.flatnonzero(keep)[:96]
    gsel = rng.choice([-1.0, 1.0], size=(len(sel), 3))
    G = np.zeros((3, H, W), np.float32)
    G[:, py[sel], px[sel]] = gsel.T
    lam = cfg.lambda_reg
    qg.qg_render_decode_bwd(n, f.ld, f.prev, f.lat, 8, f.W1, f.W2, 32, 56, f.lp, f.a, *hp, lam, cfg.sh_degree,
                            r.qcams, r.tile, cfg.dilation, r.t_proj, r.vals, r.ranges, r.bg, r.t_tf, r.t_last,
                            [to_dev(G)], f.grads["lat"], f.grads["W1"], f.grads["W2"], f.grads["lp"], f.grads["a"],
                            None, None, f.fws, f.fws_bytes)
    torch.cuda.synchronize()
    OR.render(attrs, cam, cfg.bg, pixels=(px[sel] + 0.5, py[sel] + 0.5), grad_image=gsel)
    (lam * lreg).backward()
    for k in ("lat", "W1", "W2", "lp", "a"):
        err = rel_l2(f.grads[k].cpu().numpy(), t[k].grad.numpy())
        assert err <= 1e-3, (k, err)


def _dense_planes(n):
    wl = synth.workload_dense(n)
    return wl, wl.scene.planes()


def test_dense_workload_fullsize_sampled_parity():
    from paper_2412_04469_amd import raster
    wl, planes = _dense_planes(1_000_000)
    n = wl.scene.n
    cams = wl.cams
    rast = raster.Rasterizer(n, cams, tile=(16, 16), bg=(0.0, 0.0, 0.0), capacity=1 << 24)
    attrs = to_dev(planes)
    rast.forward(attrs)  # grows the pair capacity and re-bins if needed
    torch.cuda.synchronize()
    P = int(rast.num_pairs.item())
    assert 0 < P <= rast.capacity
    rng = np.random.default_rng(11)
    tp = torch.tensor(planes.astype(np.float64), requires_grad=True)
    Gs = [torch.zeros(3, c.height, c.width, device="cuda") for c in cams]
    for v in (0, 2):
        cam = cams[v]
        px, py = _candidates(rng, cam, 96)
        ref = OR.render(tp.detach(), cam, (0.0, 0.0, 0.0), pixels=(px + 0.5, py + 0.5))
        keep = _keep(ref)
        assert keep.mean() > 0.9, keep.mean()
        assert ref["n_contrib"][keep].mean() > 30  # dense overlap reaches many contributors per pixel
        got = rast.images[v].cpu().numpy()[:, py, px].T
        assert np.abs(got - ref["color"])[keep].max() <= 1e-4
        sel = np.flatnonzero(keep)[:32]
        gsel = rng.choice([-1.0, 1.0], size=(len(sel), 3))
        Gs[v][:, py[sel], px[sel]] = torch.tensor(gsel.T, dtype=torch.float32, device="cuda")
        OR.render(tp, cam, (0.0, 0.0, 0.0), pixels=(px[sel] + 0.5, py[sel] + 0.5), grad_image=gsel)
    g = torch.zeros_like(attrs)
    rast.backward(attrs, Gs, g)
    torch.cuda.synchronize()
    gg, gr = _groups(g.cpu().numpy()), _groups(tp.grad.numpy())
    for k in gg:
        assert rel_l2(gg[k], gr[k]) <= 1e-3, (k, rel_l2(gg[k], gr[k]))


def test_dense_subscene_whole_image_gradients():
    from paper_2412_04469_amd import raster
    wl = synth.workload_dense_subscene()
    planes = wl.scene.planes()
    cam = wl.cams[0]
    rast = raster.Rasterizer(wl.scene.n, [cam], tile=(16, 16))
    attrs = to_dev(planes)
    rast.forward(attrs)
    torch.cuda.synchronize()
    ref0 = OR.render(planes.astype(np.float64), cam)
    keep = _keep(ref0)
    assert keep.mean() > 0.97
    assert np.abs(rast.images[0].cpu().numpy() - ref0["image"])[:, keep].max() <= 1e-4
    rng = np.random.default_rng(3)
    G = rng.normal(size=(3, cam.height, cam.width)) / (3 * cam.width * cam.height)
    G[:, ~keep] = 0.0
    G = G.astype(np.float32)
    tp = torch.tensor(planes.astype(np.float64), requires_grad=True)
    OR.render(tp, cam, grad_image=G.astype(np.float64))
    g = torch.zeros_like(attrs)
    rast.backward(attrs, [to_dev(G)], g)
    torch.cuda.synchronize()
    gg, gr = _groups(g.cpu().numpy()), _groups(tp.grad.numpy())
    for k in gg:
        assert rel_l2(gg[k], gr[k]) <= 1e-3, (k, rel_l2(gg[k], gr[k]))


def test_batched_workload_fullsize_sampled_parity():
    """The 12-view batched step at full size (500 k Gaussians; views at 1352x1014, 1920x1080 and 960x540) in the
    launch configuration the benchmark times (one fused decode+projection, one binning, one blend and one fused
    adjoint for all twelve views): sampled pixels of one view of each resolution against the oracle, and the
    residual-parameter gradients of a sparse image gradient spread over those three views."""
    from paper_2412_04469_amd import qg
    from paper_2412_04469_amd.fit import BatchedFitter, FitConfig
    wl = synth.workload_batched()
    n = wl.scene.n
    cfg = FitConfig()
    rng = np.random.default_rng(17)
    prev = wl.scene.planes()
    lat = rng.normal(0, 1.0, (8, n)).astype(np.float32)
    lp = rng.normal(0, 0.01, (3, n)).astype(np.float32)
    a = rng.normal(0, 1.0, n).astype(np.float32)
    gts = [torch.zeros(3, c.height, c.width, device="cuda") for c in wl.cams]
    f = BatchedFitter(to_dev(prev), wl.cams, gts, cfg, heaviest_first=False, graph=False)
    assert len(f.groups) == 1 and len(f.groups[0]) == 12
    f.lat.copy_(to_dev(lat))
    f.lp.copy_(to_dev(lp))
    f.a.copy_(to_dev(a))
    f.size_capacity()
    r = f.rasts[0]
    hp = (cfg.gamma0, cfg.gamma1, cfg.tau)
    qg.qg_decode_project(n, f.ld, f.prev, f.lat, 8, f.W1, f.W2, 32, 56, f.lp, f.a, *hp, cfg.sh_degree, r.qcams, r.tile,
                         cfg.dilation, r.t_proj, f.attrs, f.gate, None)
    r.bin()
    assert not r.overflowed()
    r.render()
    torch.cuda.synchronize()
    t = {k: torch.tensor(v.astype(np.float64), requires_grad=True)
         for k, v in (("lat", lat), ("W1", f.W1.cpu().numpy()), ("W2", f.W2.cpu().numpy()), ("lp", lp), ("a", a))}
    attrs, _, lreg = OD.decode(torch.tensor(prev.astype(np.float64)), t["lat"], t["W1"], t["W2"], t["lp"], t["a"], *hp)
    Gs = [torch.zeros(3, c.height, c.width, device="cuda") for c in wl.cams]
    picks = []
    for v in (0, 1, 3):  # 1352x1014, 1920x1080, 960x540
        cam = wl.cams[v]
        px, py = _candidates(rng, cam, 160)
        ref = OR.render(attrs.detach(), cam, cfg.bg, pixels=(px + 0.5, py + 0.5))
        keep = _keep(ref)
        print(f"view {v} ({cam.width}x{cam.height}): {int((~keep).sum())} of {keep.size} sampled pixels excluded")
        assert keep.mean() > 0.95, keep.mean()
        got = r.images[v].cpu().numpy()[:, py, px].T
        assert np.abs(got - ref["color"])[keep].max() <= 1e-4
        assert np.abs(r.tfinal[v].cpu().numpy()[py, px] - ref["t_final"])[keep].max() <= 1e-4
        sel = np.flatnonzero(keep)[:48]
        gsel = rng.choice([-1.0, 1.0], size=(len(sel), 3))
        Gs[v][:, py[sel], px[sel]] = torch.tensor(gsel.T, dtype=torch.float32, device="cuda")
        picks.append((cam, px[sel], py[sel], gsel))
    lam = cfg.lambda_reg
    qg.qg_render_decode_bwd(n, f.ld, f.prev, f.lat, 8, f.W1, f.W2, 32, 56, f.lp, f.a, *hp, lam, cfg.sh_degree,
                            r.qcams, r.tile, cfg.dilation, r.t_proj, r.vals, r.ranges, r.bg, r.t_tf, r.t_last, Gs,
                            f.grads["lat"], f.grads["W1"], f.grads["W2"], f.grads["lp"], f.grads["a"], None, None,
                            f.fws, f.fws_bytes, attrs=f.attrs)
    torch.cuda.synchronize()
    leaf = attrs.detach().clone().requires_grad_(True)  # the three views' gradients, then one pass through decode
    for cam, px, py, gsel in picks:
        OR.render(leaf, cam, cfg.bg, pixels=(px + 0.5, py + 0.5), grad_image=gsel)
    ((attrs * leaf.grad).sum() + lam * lreg).backward()
    for k in ("lat", "W1", "W2", "lp", "a"):
        err = rel_l2(f.grads[k].cpu().numpy(), t[k].grad.numpy())
        assert err <= 1e-3, (k, err)
