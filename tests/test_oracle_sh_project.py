"""Pins of the oracle's SH basis and EWA projection against closed forms, quadrature and invariants."""
import math

import numpy as np
import pytest
import torch

from oracle import project as P
from oracle import sh as SH
from paper_2412_04469_amd import synth


def _quadrature(n_theta=24, n_phi=48):
    z, w = np.polynomial.legendre.leggauss(n_theta)
    phi = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    Z, PHI = np.meshgrid(z, phi, indexing="ij")
    W = np.repeat(w[:, None], n_phi, 1) * (2 * math.pi / n_phi)
    s = np.sqrt(1 - Z * Z)
    d = np.stack([s * np.cos(PHI), s * np.sin(PHI), Z], -1).reshape(-1, 3)
    return torch.tensor(d), W.ravel()


def test_sh_orthonormal_quadrature():
    d, w = _quadrature()
    Y = SH.basis(d, 3).numpy()
    G = (Y * w[:, None]).T @ Y
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_sh_closed_form_values():
    d = torch.tensor([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]], dtype=torch.float64)
    Y = SH.basis(d, 1).numpy()
    c0 = 1.0 / (2.0 * math.sqrt(math.pi))
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    # Condon-Shortley phase: Y_1^1 = -c1 x, Y_1^-1 = -c1 y, Y_1^0 = c1 z
    np.testing.assert_allclose(Y[:, 0], c0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Y[0, 3], -c1, atol=1e-15)
    np.testing.assert_allclose(Y[1, 1], -c1, atol=1e-15)
    np.testing.assert_allclose(Y[2, 2], c1, atol=1e-15)
    np.testing.assert_allclose(Y[2, [1, 3]], 0.0, atol=1e-15)


def test_sh_addition_theorem():
    """sum_m Y_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a.b), with textbook P_0..P_3."""
    rng = np.random.default_rng(7)
    a = rng.normal(size=(50, 3)); a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = rng.normal(size=(50, 3)); b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya = SH.basis(torch.tensor(a), 3).numpy()
    Yb = SH.basis(torch.tensor(b), 3).numpy()
    x = (a * b).sum(1)
    P = [np.ones_like(x), x, (3 * x * x - 1) / 2, (5 * x ** 3 - 3 * x) / 2]
    for l in range(4):
        sl = slice(l * l, (l + 1) * (l + 1))
        lhs = (Ya[:, sl] * Yb[:, sl]).sum(1)
        np.testing.assert_allclose(lhs, (2 * l + 1) / (4 * math.pi) * P[l], atol=1e-13)


def _one(mean, quat, log_s, logit=0.0, sh=None):
    sh = np.zeros((1, 16, 3)) if sh is None else sh
    return [torch.tensor(np.asarray(v, np.float64).reshape(shape)) for v, shape in
            ((mean, (1, 3)), (quat, (1, 4)), (log_s, (1, 3)), ([logit], (1,)), (sh, (1, 16, 3)))]


def _cam(R=np.eye(3), t=np.zeros(3), f=(300.0, 200.0), c=(64.0, 48.0), w=128, h=96):
    return synth.Camera(f[0], f[1], c[0], c[1], np.asarray(R, np.float32), np.asarray(t, np.float32), w, h, 0.2)


@pytest.mark.parametrize("h", [0.0, 0.3])
def test_projection_on_axis_closed_form(h):
    s = np.array([0.05, 0.02, 0.7])
    z0 = 3.0
    cam = _cam()
    pr = P.project(*_one([0, 0, z0], [1, 0, 0, 0], np.log(s)), cam, 3, h)
    a, b, c = pr["cov2d"][0].numpy()
    np.testing.assert_allclose([a, b, c], [(cam.fx * s[0] / z0) ** 2 + h, 0.0, (cam.fy * s[1] / z0) ** 2 + h],
                               rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(pr["xy"][0].numpy(), [cam.cx, cam.cy], atol=1e-13)
    det = a * c - b * b
    np.testing.assert_allclose(pr["conic"][0].numpy(), [c / det, -b / det, a / det], rtol=1e-13)


def test_projection_off_axis_closed_form():
    s = np.array([0.05, 0.03, 0.4])
    x, z = 0.6, 2.5
    cam = _cam()
    pr = P.project(*_one([x, 0, z], [1, 0, 0, 0], np.log(s)), cam, 3, 0.0)
    a = pr["cov2d"][0, 0].item()
    np.testing.assert_allclose(a, (cam.fx / z) ** 2 * (s[0] ** 2 + (x / z) ** 2 * s[2] ** 2), rtol=1e-13)
    np.testing.assert_allclose(pr["xy"][0].numpy(), [cam.fx * x / z + cam.cx, cam.cy], rtol=1e-13)
    np.testing.assert_allclose(pr["depth"][0].item(), z, rtol=1e-15)


def test_quaternion_rotation_swaps_axes():
    """A 90 degree turn about z maps diag(sx^2, sy^2, sz^2) to diag(sy^2, sx^2, sz^2)."""
    s = np.array([0.1, 0.3, 0.2])
    q = np.array([math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)]) * 3.0  # unnormalised storage
    S = P.covariance(torch.tensor(q[None]), torch.tensor(np.log(s)[None]))[0].numpy()
    np.testing.assert_allclose(S, np.diag([s[1] ** 2, s[0] ** 2, s[2] ** 2]), atol=1e-15)


def test_ewa_matches_projected_sample_covariance():
    """Project samples of N(p, Sigma) exactly; their covariance tends to Sigma' - hI (first-order EWA)."""
    rng = np.random.default_rng(3)
    mean = np.array([0.4, -0.3, 4.0])
    q = rng.normal(size=4)
    s = np.array([0.01, 0.006, 0.015])
    cam = _cam()
    pr = P.project(*_one(mean, q, np.log(s)), cam, 3, 0.0)
    a, b, c = pr["cov2d"][0].numpy()
    Sig = P.covariance(torch.tensor(q[None]), torch.tensor(np.log(s)[None]))[0].numpy()
    X = rng.multivariate_normal(mean, Sig, size=1_000_000)
    uvx = cam.fx * X[:, 0] / X[:, 2] + cam.cx
    uvy = cam.fy * X[:, 1] / X[:, 2] + cam.cy
    emp = np.cov(np.stack([uvx, uvy]))
    np.testing.assert_allclose([emp[0, 0], emp[0, 1], emp[1, 1]], [a, b, c], rtol=2e-2, atol=2e-2 * a)


def _rot(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_rigid_motion_invariance():
    """Moving world and camera together leaves p', Sigma', depth and opacity unchanged."""
    rng = synth.rng_for(100)
    sc = synth.draw_scene(rng, 200, 0.5, -3.0, 0.4)
    cam = synth.make_camera((0.3, -0.2, -4.0), 96, 80, f=90)
    ang = 0.7
    axis = np.array([0.3, 1.0, -0.4]); axis /= np.linalg.norm(axis)
    Q = _rot(axis, ang)
    qQ = np.r_[math.cos(ang / 2), math.sin(ang / 2) * axis]
    sft = np.array([0.5, -1.0, 2.0])
    m = sc.means.astype(np.float64)
    q = sc.quats.astype(np.float64)
    base = P.project(*[torch.tensor(np.asarray(v, np.float64)) for v in (m, q, sc.log_scales, sc.logits, sc.sh)],
                     cam, 3, 0.3)
    m2 = m @ Q.T + sft
    q2 = np.stack([_qmul(qQ, qi) for qi in q])
    R2 = cam.R.astype(np.float64) @ Q.T
    t2 = cam.t.astype(np.float64) - R2 @ sft
    cam2 = synth.Camera(cam.fx, cam.fy, cam.cx, cam.cy, R2, t2, cam.width, cam.height, cam.z_near)
    # keep float64 camera (no float32 cast) for a tight check
    moved = P.project(*[torch.tensor(np.asarray(v, np.float64)) for v in (m2, q2, sc.log_scales, sc.logits, sc.sh)],
                      cam2, 3, 0.3)
    for k in ("xy", "cov2d", "depth", "opacity"):
        np.testing.assert_allclose(moved[k].numpy(), base[k].numpy(), rtol=1e-9, atol=1e-9)


def test_degree0_colour_closed_form():
    h0 = np.zeros((1, 16, 3)); h0[0, 0] = [0.3, -2.0, 0.0]
    pr = P.project(*_one([0, 0, 3], [1, 0, 0, 0], np.log([0.1] * 3), sh=h0), _cam(), 0, 0.3)
    c0 = 1 / (2 * math.sqrt(math.pi))
    np.testing.assert_allclose(pr["rgb"][0].numpy(), [0.3 * c0 + 0.5, 0.0, 0.5], atol=1e-15)


def test_culling():
    cam = _cam()
    pr = P.project(*_one([0, 0, 0.1], [1, 0, 0, 0], np.log([0.1] * 3)), cam, 3, 0.3)
    assert not bool(pr["valid"][0])
    pr = P.project(*_one([0, 0, 2.0], [1, 0, 0, 0], np.log([0.1] * 3), logit=-7.0), cam, 3, 0.3)
    assert not bool(pr["valid"][0])  # sigmoid(-7) < 1/255
    pr = P.project(*_one([0, 0, 2.0], [1, 0, 0, 0], np.log([0.1] * 3), logit=-5.0), cam, 3, 0.3)
    assert bool(pr["valid"][0])


def _pose(centre, axis, ang):
    """World->camera (R, t) of a camera at ``centre`` rotated by ``ang`` about ``axis`` (t = -R centre)."""
    R = _rot(axis, ang)
    return R, -R @ np.asarray(centre, np.float64)


# Textbook real SH with the Condon-Shortley phase, written out per (l, m) on a unit vector (x, y, z):
# index k = l^2 + l + m.
_SH_TEXTBOOK = {
    1: lambda x, y, z: -math.sqrt(3 / (4 * math.pi)) * y,                             # Y_1^-1
    2: lambda x, y, z: math.sqrt(3 / (4 * math.pi)) * z,                              # Y_1^0
    3: lambda x, y, z: -math.sqrt(3 / (4 * math.pi)) * x,                             # Y_1^1
    4: lambda x, y, z: 0.5 * math.sqrt(15 / math.pi) * x * y,                         # Y_2^-2
    6: lambda x, y, z: 0.25 * math.sqrt(5 / math.pi) * (3 * z * z - 1),               # Y_2^0
    9: lambda x, y, z: -0.25 * math.sqrt(35 / (2 * math.pi)) * (3 * x * x - y * y) * y,  # Y_3^-3
    12: lambda x, y, z: 0.25 * math.sqrt(7 / math.pi) * (5 * z ** 3 - 3 * z),          # Y_3^0
}


@pytest.mark.parametrize("k", sorted(_SH_TEXTBOOK))
def test_sh_colour_along_camera_to_mean_direction(k):
    """Colour of one SH coefficient set, for a camera that is rotated and translated: c = max(0, h Y_k(dir) + 0.5)
    with dir the unit vector from the camera centre -R^T t to the mean.  The odd degrees change sign if the
    direction is reversed, and the value depends on the camera centre, not on the camera's axis."""
    centre = np.array([0.7, -1.2, 2.0])
    R, t = _pose(centre, [0.3, 1.0, -0.4], 0.9)
    cam = _cam(R=R, t=t)
    fwd = R.T @ np.array([0.3, 0.3, 1.0])  # off the optical axis, in front of the camera
    u = fwd / np.linalg.norm(fwd)
    mean = centre + 3.0 * u
    l = int(math.isqrt(k))
    h = np.zeros((1, 16, 3)); h[0, k] = [0.8, -0.6, 1.7]
    # float64 camera: synth.Camera keeps what it is given
    cam = synth.Camera(cam.fx, cam.fy, cam.cx, cam.cy, R, t, cam.width, cam.height, cam.z_near)
    pr = P.project(*_one(mean, [1, 0, 0, 0], np.log([0.05] * 3), sh=h), cam, 3, 0.3)
    assert bool(pr["valid"][0])
    y = _SH_TEXTBOOK[k](*u)
    assert abs(y) > 0.05  # the pin is informative
    want = np.maximum(0.0, h[0, k] * y + 0.5)
    np.testing.assert_allclose(pr["rgb_pre"][0].numpy(), h[0, k] * y + 0.5, atol=1e-12)
    np.testing.assert_allclose(pr["rgb"][0].numpy(), want, atol=1e-12)
    if l % 2 == 1:
        flipped = h[0, k] * _SH_TEXTBOOK[k](*(-u)) + 0.5
        assert np.abs(flipped - (h[0, k] * y + 0.5)).max() > 0.05
    # a lower degree ignores the coefficient
    pr0 = P.project(*_one(mean, [1, 0, 0, 0], np.log([0.05] * 3), sh=h), cam, l - 1, 0.3)
    np.testing.assert_allclose(pr0["rgb"][0].numpy(), 0.5, atol=1e-15)


def _iso_splat(cx, cy, w=80, h=72):
    """sigma' = 4 px isotropic with no dilation (f s / z = 64 * 0.125 / 2), opacity 1/2, centred at (cx, cy)."""
    cam = _cam(f=(64.0, 64.0), c=(cx, cy), w=w, h=h)
    pr = P.project(*_one([0, 0, 2.0], [1, 0, 0, 0], np.log([0.125] * 3), logit=0.0), cam, 0, 0.0)
    return pr, cam


@pytest.mark.parametrize("tile,want", [((8, 8), (2, 2, 6, 6)), ((16, 16), (1, 1, 3, 3)), ((32, 8), (0, 2, 2, 6))])
def test_rectangle_exact_for_isotropic_splat(tile, want):
    """alpha >= 1/255 holds exactly on the disc of radius 4 sqrt(2 ln 127.5) = 12.4555 px; centred on the pixel
    centre (32.5, 32.5) its covered pixel columns and rows are 20..44, so the tile rectangle is known exactly.
    A rectangle one tile too large or too small fails."""
    pr, cam = _iso_splat(32.5, 32.5)
    np.testing.assert_allclose(pr["cov2d"][0].numpy(), [16.0, 0.0, 16.0], rtol=1e-14, atol=1e-14)
    j0, j1, i0, i1, empty, _ = P.pixel_rect(pr["xy"].numpy(), pr["cov2d"].numpy(), pr["opacity"].numpy(),
                                            pr["valid"].numpy(), cam.width, cam.height)
    assert (int(j0[0]), int(j1[0]), int(i0[0]), int(i1[0]), bool(empty[0])) == (20, 44, 20, 44, False)
    rect, nt, _ = P.tile_rect(pr["xy"].numpy(), pr["cov2d"].numpy(), pr["opacity"].numpy(), pr["valid"].numpy(),
                              cam.width, cam.height, *tile)
    assert tuple(int(v) for v in rect[0]) == want
    assert int(nt[0]) == (want[2] - want[0]) * (want[3] - want[1])
    # the covered pixels found by brute force span exactly those columns and rows (489 of them)
    jj, ii = np.meshgrid(np.arange(cam.width) + 0.5, np.arange(cam.height) + 0.5)
    q = ((jj - 32.5) ** 2 + (ii - 32.5) ** 2) / 16.0
    hit = np.argwhere(0.5 * np.exp(-0.5 * q) >= 1 / 255)
    assert len(hit) == 489
    assert (hit[:, 1].min(), hit[:, 1].max(), hit[:, 0].min(), hit[:, 0].max()) == (20, 44, 20, 44)


def test_rectangle_exact_clipped_and_offscreen():
    """The same splat at (5.5, 60.5) in an 80 x 72 image: columns 0..17 and rows 48..71 after clipping, 16 x 16
    tiles (0, 3)-(2, 5).  Entirely off-screen: an empty rectangle and no tiles."""
    pr, cam = _iso_splat(5.5, 60.5)
    args = (pr["xy"].numpy(), pr["cov2d"].numpy(), pr["opacity"].numpy(), pr["valid"].numpy(), cam.width, cam.height)
    j0, j1, i0, i1, empty, _ = P.pixel_rect(*args)
    assert (int(j0[0]), int(j1[0]), int(i0[0]), int(i1[0]), bool(empty[0])) == (0, 17, 48, 71, False)
    rect, nt, _ = P.tile_rect(*args, 16, 16)
    assert tuple(int(v) for v in rect[0]) == (0, 3, 2, 5) and int(nt[0]) == 4
    pr, cam = _iso_splat(-13.0, 30.0)  # support reaches x = -0.54 < 0: no pixel centre
    args = (pr["xy"].numpy(), pr["cov2d"].numpy(), pr["opacity"].numpy(), pr["valid"].numpy(), cam.width, cam.height)
    rect, nt, _ = P.tile_rect(*args, 16, 16)
    assert (rect[0] == 0).all() and int(nt[0]) == 0


def test_rectangle_tight_against_sampled_support_ellipse():
    """Tightness on a random scene: the support ellipse d^T conic d <= 2 ln(255 o) is traced as d = k L (cos t,
    sin t) with L L^T = Sigma' (Cholesky), and its sampled extent gives the pixel-centre columns and rows and the
    tiles; the oracle's rectangles must equal them (cases within 1e-3 px of a pixel-centre boundary skipped)."""
    rng = synth.rng_for(201)
    sc = synth.draw_scene(rng, 400, 1.0, -3.0, 0.6)
    cam = synth.make_camera((0.2, -0.1, -4.0), 120, 90, f=110)
    pr = P.project(*P.scene_tensors(sc), cam)
    xy, cov, o, valid = (pr[k].detach().numpy() for k in ("xy", "cov2d", "opacity", "valid"))
    ts = np.linspace(0.0, 2 * math.pi, 1 << 15, endpoint=False)
    circ = np.stack([np.cos(ts), np.sin(ts)])
    for tw, th in ((8, 8), (16, 16), (32, 8)):
        rect, nt, _ = P.tile_rect(xy, cov, o, valid, cam.width, cam.height, tw, th)
        checked = 0
        for i in np.flatnonzero(valid):
            S = np.array([[cov[i, 0], cov[i, 1]], [cov[i, 1], cov[i, 2]]])
            k = math.sqrt(2 * math.log(255 * o[i]))
            pts = k * (np.linalg.cholesky(S) @ circ)
            lo_x, hi_x = xy[i, 0] + pts[0].min(), xy[i, 0] + pts[0].max()
            lo_y, hi_y = xy[i, 1] + pts[1].min(), xy[i, 1] + pts[1].max()
            edges = np.array([lo_x - 0.5, hi_x - 0.5, lo_y - 0.5, hi_y - 0.5])
            if (np.abs(edges - np.round(edges)) < 1e-3).any():
                continue
            j0, j1 = max(math.ceil(edges[0]), 0), min(math.floor(edges[1]), cam.width - 1)
            i0, i1 = max(math.ceil(edges[2]), 0), min(math.floor(edges[3]), cam.height - 1)
            if j0 > j1 or i0 > i1:
                assert int(nt[i]) == 0 and (rect[i] == 0).all()
                continue
            assert tuple(int(v) for v in rect[i]) == (j0 // tw, i0 // th, j1 // tw + 1, i1 // th + 1), i
            checked += 1
        assert checked > 100
