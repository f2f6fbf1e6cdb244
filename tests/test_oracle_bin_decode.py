"""Pins of the oracle's binning, support rectangle, decode/gate, d_t, gate init, loss and Adam."""
import math

import numpy as np
import pytest
import torch

from oracle import adam as A
from oracle import binning as B
from oracle import composite as C
from oracle import decode as D
from oracle import gate as G
from oracle import loss as L
from oracle import project as P
from oracle import render as R
from paper_2412_04469_amd import synth


def _rand_rects(rng, n, gw, gh):
    x0 = rng.integers(0, gw, n); y0 = rng.integers(0, gh, n)
    x1 = np.minimum(x0 + rng.integers(0, 4, n), gw); y1 = np.minimum(y0 + rng.integers(0, 4, n), gh)
    return np.stack([x0, y0, x1, y1], 1).astype(np.int32)


def test_binning_matches_per_tile_brute_force():
    rng = np.random.default_rng(5)
    n, gw, gh = 400, 9, 7
    rect = _rand_rects(rng, n, gw, gh)
    depth = rng.uniform(0.5, 5, n).astype(np.float32)
    depth[::7] = depth[3]  # ties broken by index
    k1, v1 = B.make_pairs(rect, depth, gw)
    k2, v2 = B.make_pairs_fast(rect, depth, gw)
    assert np.array_equal(k1, k2) and np.array_equal(v1, v2)
    keys, vals, ranges = B.bin_view(rect, depth, gw, gh)
    bits = depth.view(np.uint32)
    for ty in range(gh):
        for tx in range(gw):
            t = ty * gw + tx
            cov = [i for i in range(n) if rect[i, 0] <= tx < rect[i, 2] and rect[i, 1] <= ty < rect[i, 3]]
            cov.sort(key=lambda i: (int(bits[i]), i))
            s, e = ranges[t]
            assert list(vals[s:e]) == cov
            assert all(int(k) >> 32 == t for k in keys[s:e])
            if not cov:
                assert s == 0 and e == 0


def test_rectangle_holds_every_covered_pixel():
    """Tiled compositing equals per-pixel compositing iff every pixel with alpha >= 1/255 lies in a tile of the
    splat's rectangle.  Checked by brute force over all pixels of a small scene."""
    rng = synth.rng_for(200)
    sc = synth.draw_scene(rng, 300, 1.0, -3.0, 0.5)
    cam = synth.make_camera((0.0, 0.0, -4.0), 80, 64, f=80)
    pr = P.project(*P.scene_tensors(sc), cam)
    tw, th = 8, 8
    rect, ntiles, _ = P.tile_rect(pr["xy"].numpy(), pr["cov2d"].numpy(), pr["opacity"].numpy(),
                                  pr["valid"].numpy(), cam.width, cam.height, tw, th)
    jj, ii = np.meshgrid(np.arange(cam.width) + 0.5, np.arange(cam.height) + 0.5)
    xy, con, o = pr["xy"].numpy(), pr["conic"].numpy(), pr["opacity"].numpy()
    seen = 0
    for i in np.flatnonzero(pr["valid"].numpy()):
        dx = jj - xy[i, 0]; dy = ii - xy[i, 1]
        a = np.minimum(0.99, o[i] * np.exp(-0.5 * (con[i, 0] * dx * dx + 2 * con[i, 1] * dx * dy + con[i, 2] * dy * dy)))
        hit = np.argwhere(a >= 1 / 255)
        for (r_, c_) in hit:
            tx, ty = c_ // tw, r_ // th
            assert rect[i, 0] <= tx < rect[i, 2] and rect[i, 1] <= ty < rect[i, 3]
        seen += len(hit)
        if len(hit) == 0:
            continue
    assert seen > 1000
    assert (ntiles[~pr["valid"].numpy()] == 0).all()


N3DV = (-0.5, 1.01, 0.3)
IMM = (-0.1, 1.1, 0.5)


def test_gate_closed_forms_n3dv():
    g0, g1, tau = N3DV
    a = torch.tensor([0.0], dtype=torch.float64, requires_grad=True)
    g = D.gate(a, g0, g1, tau)
    np.testing.assert_allclose(g.item(), 0.255, atol=1e-15)
    g.backward()
    np.testing.assert_allclose(a.grad.item(), (g1 - g0) / (4 * tau), rtol=1e-14)
    np.testing.assert_allclose(a.grad.item(), 1.2583333, atol=1e-7)
    closing = tau * math.log(-g0 / g1)
    opening = tau * math.log((1 - g0) / (g1 - 1))
    np.testing.assert_allclose([closing, opening], [-0.2109293, 1.5031906], atol=1e-7)
    t = torch.tensor([closing - 1e-9, closing + 1e-6, opening - 1e-6, opening + 1e-9], dtype=torch.float64)
    gg = D.gate(t, g0, g1, tau).numpy()
    assert gg[0] == 0.0 and 0 < gg[1] < 1e-5 and 1 - 1e-5 < gg[2] < 1.0 and gg[3] == 1.0
    p = torch.sigmoid(torch.tensor(0.0 - closing)).item()
    np.testing.assert_allclose(p, 0.5525377, atol=1e-7)


def test_gate_closed_forms_immersive():
    g0, g1, tau = IMM
    a = torch.tensor([0.0], dtype=torch.float64, requires_grad=True)
    g = D.gate(a, g0, g1, tau)
    np.testing.assert_allclose(g.item(), 0.5, atol=1e-15)
    g.backward()
    np.testing.assert_allclose(a.grad.item(), 0.6, rtol=1e-14)
    np.testing.assert_allclose(tau * math.log(-g0 / g1), -1.1989476, atol=1e-7)
    np.testing.assert_allclose(tau * math.log((1 - g0) / (g1 - 1)), 1.1989476, atol=1e-7)
    np.testing.assert_allclose(torch.sigmoid(torch.tensor(-tau * math.log(-g0 / g1))).item(), 0.7683375, atol=1e-7)


def test_rounding_and_zero_latents():
    x = torch.tensor([0.5, 1.5, -0.5, 2.5, -1.5, 0.49], dtype=torch.float64)
    r = D.ste_round(x)
    assert r.tolist() == [0.0, 2.0, -0.0, 2.0, -2.0, 0.0]
    assert math.copysign(1, torch.round(x)[2].item()) == -1  # rint(-0.5) = -0
    rng = np.random.default_rng(0)
    W1 = torch.tensor(rng.normal(size=(32, 8))); W2 = torch.tensor(rng.normal(size=(56, 32)))
    prev = torch.tensor(rng.normal(size=(59, 10)))
    out, g, _ = D.decode(prev, torch.zeros(8, 10, dtype=torch.float64) + 0.3, W1, W2, torch.zeros(3, 10, dtype=torch.float64),
                         torch.zeros(10, dtype=torch.float64), *N3DV)
    assert torch.equal(out, prev)


def test_decode_matches_torch_layers_and_ste_gradient():
    rng = np.random.default_rng(1)
    n = 50
    lat = torch.tensor(rng.normal(0, 2, size=(8, n)), requires_grad=True)
    W1 = torch.tensor(rng.normal(size=(32, 8)), requires_grad=True)
    W2 = torch.tensor(rng.normal(size=(56, 32)))
    prev = torch.tensor(rng.normal(size=(59, n)))
    lp = torch.tensor(rng.normal(size=(3, n)))
    a = torch.tensor(rng.normal(size=n))
    out, g, lreg = D.decode(prev, lat, W1, W2, lp, a, *IMM)
    ref = torch.nn.functional.linear(torch.nn.functional.silu(torch.nn.functional.linear(torch.round(lat.T), W1)), W2)
    np.testing.assert_allclose((out[3:] - prev[3:]).T.detach().numpy(), ref.detach().numpy(), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose((out[:3] - prev[:3]).detach().numpy(), (g * lp).detach().numpy(), rtol=1e-13, atol=1e-14)
    # STE: the gradient wrt latents equals the gradient wrt the rounded latents
    Gout = torch.tensor(rng.normal(size=(59, n)))
    (out * Gout).sum().backward()
    lr_ = torch.round(lat.detach().T).requires_grad_(True)
    ref2 = torch.nn.functional.linear(torch.nn.functional.silu(torch.nn.functional.linear(lr_, W1.detach())), W2)
    (ref2 * Gout[3:].T).sum().backward()
    np.testing.assert_allclose(lat.grad.T.numpy(), lr_.grad.numpy(), rtol=1e-12)
    s = D.l_reg(a, *IMM, reduction="sum")
    np.testing.assert_allclose(s.item(), lreg.item() * n, rtol=1e-14)


def test_dt_one_pass_equals_two_pass_and_static_is_zero():
    rng = synth.rng_for(300)
    sc = synth.draw_scene(rng, 150, 0.6, -3.0, 0.4)
    cam = synth.make_camera((0.0, 0.0, -3.0), 40, 32, f=40)
    planes = sc.planes().astype(np.float64)
    base = R.render(planes, cam)
    img = base["image"]
    I_prev = np.clip(img + rng.normal(0, 0.05, img.shape), 0, 1)
    I_cur = np.clip(img + rng.normal(0, 0.05, img.shape), 0, 1)
    r1 = R.render(planes, cam, grad_image=G.mse_grad(img, I_cur))
    r2 = R.render(planes, cam, grad_image=G.mse_grad(img, I_prev))
    r3 = R.render(planes, cam, grad_image=G.dt_image_gradient(I_prev, I_cur))
    two = r1["g_xy"] - r2["g_xy"]
    np.testing.assert_allclose(r3["g_xy"], two, atol=1e-12 * max(1, np.abs(two).max()))
    assert np.abs(two).max() > 0
    r0 = R.render(planes, cam, grad_image=G.dt_image_gradient(I_cur, I_cur))
    assert np.abs(r0["g_xy"]).max() == 0.0


def test_gate_init_invariants():
    rng = np.random.default_rng(4)
    d = rng.normal(size=(101, 2))
    p, a = G.gate_init(d, *N3DV)
    p2, a2 = G.gate_init(d * 37.5, *N3DV)
    np.testing.assert_allclose(a, a2, rtol=1e-12, atol=1e-12)
    nrm = np.linalg.norm(d, axis=1)
    med = np.sort(nrm)[50]
    i = int(np.flatnonzero(nrm == med)[0])
    assert p[i] == 0.5
    np.testing.assert_allclose(a[i], N3DV[2] * math.log(-N3DV[0] / N3DV[1]), atol=1e-15)
    # Eq. 8's probability recovers p
    np.testing.assert_allclose(torch.sigmoid(torch.tensor(a - N3DV[2] * math.log(-N3DV[0] / N3DV[1]))).numpy(), p, rtol=1e-12)
    pz, _ = G.gate_init(np.zeros((5, 2)), *N3DV)
    assert (pz == 1e-6).all()


def test_l1_and_psnr_closed_forms():
    I = np.random.default_rng(0).uniform(size=(3, 4, 5))
    v, g = L.l1(I, I)
    assert v == 0.0 and (g == 0).all()
    J = I.copy(); J[0, 0, 0] += 0.5; J[1, 1, 1] -= 0.25
    v, g = L.l1(J, I)
    np.testing.assert_allclose(v, 0.75 / 60, rtol=1e-15)
    assert g[0, 0, 0] == 1 / 60 and g[1, 1, 1] == -1 / 60 and np.count_nonzero(g) == 2
    gt = np.full((3, 10, 10), 0.5)
    np.testing.assert_allclose(L.psnr(gt + 0.01, gt), 40.0, rtol=1e-12)


def test_adam_matches_torch():
    rng = np.random.default_rng(9)
    th = rng.normal(size=20)
    t_th = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([t_th], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(20); v = np.zeros(20)
    for step in range(1, 6):
        g = rng.normal(size=20)
        t_th.grad = torch.tensor(g)
        opt.step()
        th, m, v = A.adam_step(th, g, m, v, step, 0.05)
    np.testing.assert_allclose(th, t_th.detach().numpy(), rtol=1e-13, atol=1e-14)


def test_paper_mode_linear_decoder():
    """Eq. 5 as written: r_c = D_c rint(l_c) per category, the quantisation table's latent dimensions; pinned by
    torch.nn.functional.linear per block, the block structure (a category's latents move only its own planes),
    zero latents -> zero residual, and the straight-through gradient."""
    import torch.nn.functional as F
    dims = D.PAPER_DIMS_N3DV
    assert sum(dims) == 29 and sum(D.PAPER_DIMS_IMMERSIVE) == 37
    assert [m for _, _, m in D.PAPER_CATEGORIES] == [4, 3, 1, 3, 45]
    assert [p for _, p, _ in D.PAPER_CATEGORIES] == [3, 7, 10, 11, 14]
    rng = np.random.default_rng(3)
    n = 50
    lat = torch.tensor(rng.normal(0, 2, size=(29, n)), requires_grad=True)
    Ds = [torch.tensor(rng.normal(size=(m, L)), requires_grad=True) for (_, _, m), L in zip(D.PAPER_CATEGORIES, dims)]
    r = D.linear_decode(lat, Ds, dims)
    assert r.shape == (56, n)
    lr = torch.round(lat.detach())
    ref, k = [], 0
    for (_, _, m), L, Dc in zip(D.PAPER_CATEGORIES, dims, Ds):
        ref.append(F.linear(lr[k:k + L].T, Dc.detach()).T)
        k += L
    assert torch.allclose(r, torch.cat(ref, 0), rtol=1e-14, atol=1e-12)
    # block structure: the opacity latents (rows 14..16) move only plane 10 (row 7 of the residual)
    lat2 = lat.detach().clone()
    lat2[14:17] += 3.0
    r2 = D.linear_decode(lat2, [d.detach() for d in Ds], dims)
    diff = (r2 - r.detach()).abs().sum(1)
    assert diff[7] > 0 and diff[:7].sum() == 0 and diff[8:].sum() == 0
    assert D.linear_decode(torch.zeros(29, 4, dtype=torch.float64), Ds, dims).abs().max() == 0
    # straight-through gradients: dL/dl_c = D_c^T dL/dr_c, dL/dD_c = dL/dr_c rint(l_c)^T
    G = torch.tensor(rng.normal(size=(56, n)))
    (r * G).sum().backward()
    k, row = 0, 0
    for (_, _, m), L, Dc in zip(D.PAPER_CATEGORIES, dims, Ds):
        assert torch.allclose(lat.grad[k:k + L], Dc.detach().T @ G[row:row + m], rtol=1e-12)
        assert torch.allclose(Dc.grad, G[row:row + m] @ lr[k:k + L].T, rtol=1e-12)
        k += L
        row += m
