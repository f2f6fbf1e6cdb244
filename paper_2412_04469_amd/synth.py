"""Seeded synthetic inputs: Gaussian scenes, camera rigs, per-frame motion.

This module only draws random numbers and builds camera poses.  It holds none
of the method's arithmetic (no projection, no blending, no decoding) so that the
HIP path and the CPU oracle can both be fed from it without sharing code.

Every draw is made in float64 by ``numpy.random.Generator(PCG64(SeedSequence(
[2412, 4469, k])))`` in a fixed order and then cast to float32, so both sides of
a parity test receive identical float32 arrays.

Scene statistics follow the workloads the paper trains on (Sec. 3.1: Gaussians
with mean, quaternion, scale, opacity and SH colour; Sec. 4.1 and App. C: 20-view
forward-facing rigs at 1352x1014 with the central view held out, SH degree 3 for
the Immersive setting).  The public datasets themselves are not available, so
these draws stand in for them.

Attribute plane layout (float32, SoA ``[59][N]``):
    0-2   mean x, y, z
    3-6   quaternion w, x, y, z (unnormalised storage)
    7-9   log-scale x, y, z
    10    opacity logit
    11+3k+ch  SH coefficient of basis k (0..15), colour channel ch (0..2)
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

N_PLANES = 59
SH_COEFFS = 16


def rng_for(k: int) -> np.random.Generator:
    """Generator for workload k (``SeedSequence([2412, 4469, k])``)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([2412, 4469, int(k)])))


@dataclasses.dataclass
class Scene:
    """Named float32 attribute arrays of N Gaussians."""
    means: np.ndarray       # [N,3]
    quats: np.ndarray       # [N,4] (w,x,y,z), unit length as drawn
    log_scales: np.ndarray  # [N,3]
    logits: np.ndarray      # [N]
    sh: np.ndarray          # [N,16,3]

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def planes(self) -> np.ndarray:
        """Pack into the ``[59][N]`` float32 plane layout."""
        out = np.empty((N_PLANES, self.n), np.float32)
        out[0:3] = self.means.T
        out[3:7] = self.quats.T
        out[7:10] = self.log_scales.T
        out[10] = self.logits
        out[11:] = self.sh.reshape(self.n, 48).T
        return out

    @staticmethod
    def from_planes(p: np.ndarray) -> "Scene":
        p = np.asarray(p, np.float32)
        n = p.shape[1]
        return Scene(means=np.ascontiguousarray(p[0:3].T), quats=np.ascontiguousarray(p[3:7].T),
                     log_scales=np.ascontiguousarray(p[7:10].T), logits=np.ascontiguousarray(p[10]),
                     sh=np.ascontiguousarray(p[11:].T.reshape(n, 16, 3)))

    def copy(self) -> "Scene":
        return Scene(*(np.array(a, copy=True) for a in (self.means, self.quats, self.log_scales,
                                                         self.logits, self.sh)))

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx], self.quats[idx], self.log_scales[idx], self.logits[idx], self.sh[idx])


def draw_scene(rng: np.random.Generator, n: int, mean_std: float = 1.0, log_scale_mu: float = -4.0,
               log_scale_std: float = 0.5) -> Scene:
    """Draw N Gaussians in the fixed order: means, log-scales, quaternions, logits, SH DC, SH rest."""
    means = rng.normal(0.0, mean_std, size=(n, 3))
    log_s = rng.normal(log_scale_mu, log_scale_std, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logits = rng.normal(0.0, 1.0, size=n)
    dc = rng.normal(0.0, 0.5, size=(n, 3))
    rest = rng.normal(0.0, 0.1, size=(n, 15, 3))
    sh = np.concatenate([dc[:, None, :], rest], axis=1)
    f = np.float32
    return Scene(means.astype(f), q.astype(f), log_s.astype(f), logits.astype(f), sh.astype(f))


@dataclasses.dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward), world->camera ``u = R p + t``.

    Pixel (row i, column j) has its centre at (j + 0.5, i + 0.5).
    """
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # [3,3] float32, row-major
    t: np.ndarray  # [3] float32
    width: int
    height: int
    z_near: float = 0.2

    def center(self) -> np.ndarray:
        R = self.R.astype(np.float64)
        return -R.T @ self.t.astype(np.float64)


def look_at(center, target=(0.0, 0.0, 0.0), down=(0.0, 1.0, 0.0)):
    """World->camera rotation and translation for a camera at ``center`` looking at ``target``.

    The camera's y axis is the component of ``down`` orthogonal to the viewing direction.
    """
    c = np.asarray(center, np.float64)
    z = np.asarray(target, np.float64) - c
    z /= np.linalg.norm(z)
    d = np.asarray(down, np.float64)
    y = d - z * np.dot(d, z)
    y /= np.linalg.norm(y)
    x = np.cross(y, z)
    R = np.stack([x, y, z])
    t = -R @ c
    return R.astype(np.float32), t.astype(np.float32)


def make_camera(center, width, height, f=None, target=(0.0, 0.0, 0.0), z_near=0.2) -> Camera:
    R, t = look_at(center, target)
    f = float(width if f is None else f)
    return Camera(f, f, width / 2.0, height / 2.0, R, t, int(width), int(height), float(z_near))


def arc_cameras(n_views: int, radius: float, arc_deg: float, width: int, height: int, f=None):
    """Cameras on an arc of the y = 0 plane, centre ``r (sin th, 0, -cos th)``, looking at the origin.

    ``th_k = -arc/2 + arc * k / (n_views - 1)``.
    """
    cams = []
    for k in range(n_views):
        th = math.radians(-arc_deg / 2.0 + arc_deg * k / max(1, n_views - 1))
        c = (radius * math.sin(th), 0.0, -radius * math.cos(th))
        cams.append(make_camera(c, width, height, f))
    return cams


# ----------------------------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    cams: list
    target_scene: Scene | None = None  # scene whose render is the ground truth
    tile: tuple = (16, 16)
    extras: dict = dataclasses.field(default_factory=dict)


def workload_small(n: int = 10_000, width: int = 256, height: int = 256) -> Workload:
    """10 k Gaussians, one 256x256 camera (f = 256) at distance 4 facing the origin, 16x16 tiles.

    Ground truth: the same scene with means displaced by N(0, 0.01), drawn after the scene.
    """
    rng = rng_for(0)
    sc = draw_scene(rng, n, 1.0, -4.0, 0.5)
    gt = sc.copy()
    gt.means = (sc.means.astype(np.float64) + rng.normal(0.0, 0.01, size=(n, 3))).astype(np.float32)
    cam = make_camera((0.0, 0.0, -4.0), width, height, f=width)
    return Workload("gauss10k_256x256_1view", sc, [cam], gt)


def _moved_scene(rng, sc: Scene, frac_move=0.10, frac_colour=0.05):
    n = sc.n
    gt = sc.copy()
    perm = rng.permutation(n)
    k = int(round(frac_move * n))
    mv = perm[:k]
    u = rng.normal(size=(k, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    amp = rng.uniform(0.05, 0.3, size=k)
    gt.means[mv] = (sc.means[mv].astype(np.float64) + u * amp[:, None]).astype(np.float32)
    kc = int(round(frac_colour * n))
    cc = rng.permutation(n)[:kc]
    gt.sh[cc, 0, :] = (sc.sh[cc, 0, :].astype(np.float64) + rng.normal(0.0, 0.1, size=(kc, 3))).astype(np.float32)
    return gt


def workload_fit(n: int = 300_000, width: int = 1352, height: int = 1014, n_views: int = 20) -> Workload:
    """Per-frame residual fit: 300 k Gaussians (means N(0,2)^3), 20 cameras on a 120 degree arc of radius 5,
    1352x1014, f = W, plus a held-out camera at the arc centre.  Ground-truth frame: 10% of Gaussians moved
    by u*A (u uniform on S^2, A ~ U(0.05, 0.3)) and the SH DC of 5% shifted by N(0, 0.1)."""
    rng = rng_for(1)
    sc = draw_scene(rng, n, 2.0, -4.0, 0.5)
    gt = _moved_scene(rng, sc)
    cams = arc_cameras(n_views, 5.0, 120.0, width, height)
    held = make_camera((0.0, 0.0, -5.0), width, height)
    return Workload("gauss300k_1352x1014_20view_fit", sc, cams, gt, extras={"held_out": held})


def workload_fit_local(n: int = 300_000, width: int = 1352, height: int = 1014, n_views: int = 20,
                       frac_move: float = 0.003, centre=(0.5, 0.3, -2.5)) -> Workload:
    """The per-frame fit scene and cameras of workload_fit with spatially localised change (a moving object in a
    static scene): the frac_move of the Gaussians nearest to `centre` (on the camera side of the cloud, so the
    object is visible) are moved by u*A (u uniform on S^2, A ~ U(0.05, 0.3)) and half of those also get their
    SH DC shifted by N(0, 0.1)."""
    rng = rng_for(1)
    sc = draw_scene(rng, n, 2.0, -4.0, 0.5)
    rng2 = rng_for(5)
    gt = sc.copy()
    centre = np.asarray(centre, np.float64)
    k = int(round(frac_move * n))
    dist = np.linalg.norm(sc.means.astype(np.float64) - centre, axis=1)
    mv = np.sort(np.argsort(dist, kind="stable")[:k])
    u = rng2.normal(size=(k, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    amp = rng2.uniform(0.05, 0.3, size=k)
    gt.means[mv] = (sc.means[mv].astype(np.float64) + u * amp[:, None]).astype(np.float32)
    cc = mv[rng2.permutation(k)[:k // 2]]
    gt.sh[cc, 0, :] = (sc.sh[cc, 0, :].astype(np.float64) + rng2.normal(0.0, 0.1, size=(len(cc), 3))).astype(np.float32)
    cams = arc_cameras(n_views, 5.0, 120.0, width, height)
    held = make_camera((0.0, 0.0, -5.0), width, height)
    return Workload("gauss300k_1352x1014_20view_fit_local", sc, cams, gt, extras={"held_out": held, "moved": mv})


def workload_batched(n: int = 500_000) -> Workload:
    """12 views of one timestep on the 120 degree arc at uneven resolutions: even k at 1352x1014,
    k in {1,5,7,11} at 1920x1080, k in {3,9} at 960x540; f = W per view."""
    rng = rng_for(2)
    sc = draw_scene(rng, n, 2.0, -4.0, 0.5)
    gt = _moved_scene(rng, sc)
    cams = []
    for k in range(12):
        if k % 2 == 0:
            w, h = 1352, 1014
        elif k in (1, 5, 7, 11):
            w, h = 1920, 1080
        else:
            w, h = 960, 540
        th = math.radians(-60.0 + 120.0 * k / 11)
        cams.append(make_camera((5.0 * math.sin(th), 0.0, -5.0 * math.cos(th)), w, h))
    return Workload("gauss500k_12view_uneven", sc, cams, gt)


def workload_dense(n: int = 1_000_000) -> Workload:
    """Dense overlap: 1 M Gaussians, means N(0,1)^3, log-scales N(-3, 0.5); 4 views at
    th in {-45, -15, 15, 45} degrees, radius 4, 1920x1080, f = 1920."""
    rng = rng_for(3)
    sc = draw_scene(rng, n, 1.0, -3.0, 0.5)
    gt = sc.copy()
    gt.means = (sc.means.astype(np.float64) + rng.normal(0.0, 0.01, size=(n, 3))).astype(np.float32)
    cams = []
    for deg in (-45.0, -15.0, 15.0, 45.0):
        th = math.radians(deg)
        cams.append(make_camera((4.0 * math.sin(th), 0.0, -4.0 * math.cos(th)), 1920, 1080))
    return Workload("gauss1m_1920x1080_4view_dense", sc, cams, gt)


def workload_dense_subscene() -> Workload:
    """The first 2,000 Gaussians of the dense draw, 64x64, f = 64, camera at distance 4."""
    full = workload_dense()
    idx = np.arange(2000)
    cam = make_camera((0.0, 0.0, -4.0), 64, 64, f=64)
    return Workload("gauss2k_64x64_fd", full.scene.subset(idx), [cam], full.target_scene.subset(idx))


def dynamic_motion(n: int, rng_k: int = 4, frac: float = 0.10):
    """Sinusoidal motion of 10% of the Gaussians (seeded permutation): p_i(t) = p_i + A_i sin(2 pi t / P_i + phi_i) u_i
    with u_i uniform on S^2, A_i ~ U(0.05, 0.3), P_i ~ U(10, 40) frames, phi_i ~ U(0, 2 pi).
    Returns (moving indices, u [k,3], A [k], P [k], phi [k]) in float64."""
    rng = rng_for(rng_k)
    _ = draw_scene(rng, n, 2.0, -4.0, 0.5)  # keep the stream aligned with the scene draw
    perm = rng.permutation(n)
    k = int(round(frac * n))
    mv = np.sort(perm[:k])
    u = rng.normal(size=(k, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    A = rng.uniform(0.05, 0.3, size=k)
    P = rng.uniform(10.0, 40.0, size=k)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=k)
    return mv, u, A, P, phi


def workload_dynamic(n: int = 300_000, n_views: int = 20, width: int = 1352, height: int = 1014):
    """50-frame dynamic scene (frames 0..50); the scene draw equals the per-frame fit's distributions."""
    rng = rng_for(4)
    sc = draw_scene(rng, n, 2.0, -4.0, 0.5)
    cams = arc_cameras(n_views, 5.0, 120.0, width, height)
    held = make_camera((0.0, 0.0, -5.0), width, height)
    motion = dynamic_motion(n)
    return Workload("gauss300k_50frame_dynamic", sc, cams, None, extras={"held_out": held, "motion": motion})


def frame_scene(base: Scene, motion, t: int) -> Scene:
    """The dynamic scene at frame t (positions only move)."""
    mv, u, A, P, phi = motion
    out = base.copy()
    disp = (A * np.sin(2.0 * math.pi * t / P + phi))[:, None] * u
    out.means[mv] = (base.means[mv].astype(np.float64) + disp).astype(np.float32)
    return out


def random_image(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    """Uniform [0,1) image ``[3][H][W]`` float32."""
    return rng.uniform(0.0, 1.0, size=(3, h, w)).astype(np.float32)


def random_splats(rng: np.random.Generator, n: int, width: int, height: int, radius_px=(1.0, 12.0),
                  opacity=(0.02, 0.99)):
    """2D splat records drawn directly in image space (for blend-only tests).

    Returns a dict of float32 arrays: xy [N,2], conic [N,3] (inverse covariance entries A, B, C of
    ``A dx^2 + 2 B dx dy + C dy^2``), opacity [N], rgb [N,3], depth [N]."""
    xy = np.stack([rng.uniform(-4, width + 4, n), rng.uniform(-4, height + 4, n)], 1)
    sx = rng.uniform(*radius_px, n)
    sy = rng.uniform(*radius_px, n)
    th = rng.uniform(0, math.pi, n)
    c, s = np.cos(th), np.sin(th)
    # covariance = Rot diag(sx^2, sy^2) Rot^T
    a = c * c * sx * sx + s * s * sy * sy
    b = c * s * (sx * sx - sy * sy)
    d = s * s * sx * sx + c * c * sy * sy
    det = a * d - b * b
    conic = np.stack([d / det, -b / det, a / det], 1)
    op = rng.uniform(*opacity, n)
    rgb = rng.uniform(0, 1, (n, 3))
    depth = rng.uniform(0.5, 10.0, n)
    f = np.float32
    return {"xy": xy.astype(f), "conic": conic.astype(f), "opacity": op.astype(f), "rgb": rgb.astype(f),
            "depth": depth.astype(f)}
