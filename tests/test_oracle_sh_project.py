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
