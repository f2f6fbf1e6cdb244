"""Pins of the oracle's stochastic gate (with its counter-based generator) and of per-frame densification (CPU)."""
import math
import os

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import decode as D
from oracle import densify as DS
from oracle import philox as PX

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = PX.philox4x32_10(np.array(ctr, np.uint64), np.array(key, np.uint64))
        assert [int(x) for x in got] == want


def test_uniforms_are_open_interval_and_float32_exact():
    x = np.array([0, 1, 255, 256, 0xFFFFFFFF, 0x80000000], np.uint64)
    u = PX.uniform(x)
    assert (u > 0).all() and (u < 1).all()
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    assert u[0] == 0.5 / 2 ** 23 and u[4] == 1.0 - 0.5 / 2 ** 23
    v = PX.gate_uniforms(200000, seed=123, step=7)
    assert abs(v.mean() - 0.5) < 4 * math.sqrt(1 / 12 / len(v))
    assert not np.array_equal(v, PX.gate_uniforms(200000, seed=123, step=8))  # a new draw per step


@pytest.mark.parametrize("hp", [(-0.5, 1.01, 0.3), (-0.1, 1.1, 0.5)])
def test_stochastic_gate_reduces_to_the_deterministic_one_at_u_half(hp):
    a = torch.linspace(-3, 3, 101, dtype=torch.float64)
    noise = D.logistic_noise(torch.full((101,), 0.5, dtype=torch.float64))
    assert torch.equal(noise, torch.zeros(101, dtype=torch.float64))
    assert torch.equal(D.gate(a, *hp, noise=noise), D.gate(a, *hp))


@pytest.mark.parametrize("hp", [(-0.5, 1.01, 0.3), (-0.1, 1.1, 0.5)])
@pytest.mark.parametrize("a0", [-1.0, 0.0, 0.7])
def test_stochastic_gate_is_nonzero_with_eq8_probability(hp, a0):
    """Under the hard concrete noise, P(g > 0) = sigmoid(a - tau log(-gamma0/gamma1)): Eq. 8's p_i is the
    probability that the gate is open.  Also P(g = 1) = sigmoid(a - tau log((1 - gamma0)/(gamma1 - 1)))."""
    g0, g1, tau = hp
    m = 400000
    u = PX.gate_uniforms(m, seed=99, step=3)
    g = D.gate(torch.full((m,), a0, dtype=torch.float64), *hp, noise=D.logistic_noise(u)).numpy()
    p_open = 1.0 / (1.0 + math.exp(-(a0 - tau * math.log(-g0 / g1))))
    p_one = 1.0 / (1.0 + math.exp(-(a0 - tau * math.log((1 - g0) / (g1 - 1)))))
    for frac, p in (((g > 0).mean(), p_open), ((g >= 1).mean(), p_one)):
        assert abs(frac - p) < 5 * math.sqrt(p * (1 - p) / m), (frac, p)
    lreg = D.l_reg(torch.tensor([a0], dtype=torch.float64), *hp).item()
    assert abs(lreg - p_open) < 1e-15


def test_split_normals_are_standard_normal():
    z = PX.split_normals(np.arange(100000), seed=5, rnd=2)
    assert z.shape == (100000, 6)
    assert np.abs(z.mean(0)).max() < 4 / math.sqrt(len(z))
    assert np.abs(z.var(0) - 1).max() < 4 * math.sqrt(2 / len(z))
    c = np.corrcoef(z.T)
    assert np.abs(c - np.eye(6)).max() < 4 / math.sqrt(len(z))


def test_plan_actions_hand_example():
    accum = np.array([0.0, 0.01, 0.01, 0.0026, 0.0024, 0.5, 0.01])
    count = np.array([0.0, 4.0, 4.0, 2.0, 2.0, 10.0, 4.0])  # scores 0, .0025, .0025, .0013, .0012, .05, .0025
    ls = np.log(np.array([[0.01, 0.01, 0.2, 0.01, 0.01, 0.01, 0.01]] * 3))
    logits = np.array([0.0, 0.0, 0.0, 0.0, 0.0, -6.0, 0.0])  # sigmoid(-6) = 0.0025 < 0.005: pruned
    act = DS.plan(accum, count, ls, logits, threshold=0.00125, max_scale=0.05)
    assert act.tolist() == [DS.KEEP, DS.CLONE, DS.SPLIT, DS.CLONE, DS.KEEP, DS.PRUNE, DS.CLONE]


def _state(n, rng):
    prev = rng.normal(size=(59, n))
    dec = prev + rng.normal(0, 0.1, size=(59, n))
    dec[7:10] = np.log(rng.uniform(0.01, 0.1, size=(3, n)))
    params = [rng.normal(size=(8, n)), rng.normal(size=(3, n)), rng.normal(size=(1, n))]
    moments = [rng.normal(size=(12, n)), rng.uniform(size=(12, n))]
    return prev, dec, params, moments


def test_apply_clones_splits_prunes():
    rng = np.random.default_rng(0)
    n = 9
    prev, dec, params, moments = _state(n, rng)
    act = np.array([0, 1, 2, 3, 0, 2, 1, 3, 0])
    z = rng.normal(size=(n, 6))
    npv, npar, nmom, parent = DS.apply(act, prev, dec, params, moments, seed=1, rnd=0, normals=z)
    assert len(parent) == n - 2 + 2 + 2 == 11
    assert parent.tolist() == [0, 1, 1, 2, 2, 4, 5, 5, 6, 6, 8]
    # kept Gaussians: exact copies; clones: copies apart from the opacity logit; moments on the first child only
    for j, i in enumerate(parent):
        for arr, src in zip(npar, params):
            assert np.array_equal(arr[:, j], src[:, i])
        if act[i] == DS.KEEP:
            assert np.array_equal(npv[:, j], prev[:, i])
        if act[i] == DS.CLONE:
            keep_planes = [k for k in range(59) if k != 10]
            assert np.array_equal(npv[keep_planes, j], prev[keep_planes, i])
            o = 1.0 / (1.0 + math.exp(-dec[10, i]))
            o2 = 1.0 / (1.0 + math.exp(-(dec[10, i] + npv[10, j] - prev[10, i])))
            assert abs(1.0 - (1.0 - o2) ** 2 - o) < 1e-12
    for j in (0, 1, 5, 8, 10):
        for arr, src in zip(nmom, moments):
            assert np.array_equal(arr[:, j], src[:, parent[j]])
    for j in (2, 3, 4, 6, 7, 9):
        for arr in nmom:
            assert (arr[:, j] == 0).all()
    # split children: log-scale - ln 1.6, mean offset R(q) (s * z) of the decoded parent (scipy rotation)
    for j in (3, 4, 6, 7):
        i = parent[j]
        zz = z[i, 0:3] if parent[j - 1] != i else z[i, 3:6]
        q = dec[3:7, i] / np.linalg.norm(dec[3:7, i])
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        off = R @ (np.exp(dec[7:10, i]) * zz)
        np.testing.assert_allclose(npv[0:3, j], prev[0:3, i] + off, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(npv[7:10, j], prev[7:10, i] - math.log(1.6), rtol=0, atol=1e-12)
        assert np.array_equal(npv[10:59, j], prev[10:59, i]) and np.array_equal(npv[3:7, j], prev[3:7, i])
    # z = 0 keeps the mean
    npv0, _, _, parent0 = DS.apply(act, prev, dec, params, moments, seed=1, rnd=0, normals=np.zeros((n, 6)))
    for j in np.flatnonzero(act[parent0] == DS.SPLIT):
        assert np.array_equal(npv0[0:3, j], prev[0:3, parent0[j]])


def test_quaternion_matrix_against_scipy():
    rng = np.random.default_rng(1)
    q = rng.normal(size=(50, 4))
    R = DS.quat_matrix(q)
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    ref = Rotation.from_quat(qn[:, [1, 2, 3, 0]]).as_matrix()
    np.testing.assert_allclose(R, ref, atol=1e-12)


def test_schedule_and_extent():
    # 25 epochs of 20 views: after epochs 6, 8, ..., 20 (80% of 25)
    assert DS.schedule(20, 25) == [120, 160, 200, 240, 280, 320, 360, 400]
    assert DS.camera_extent([[1, 0, 0], [-1, 0, 0], [0, 0, 0]]) == pytest.approx(1.1)


def test_accumulate_uses_ndc_units_and_visibility():
    acc, cnt = np.zeros(3), np.zeros(3)
    g = np.array([[3.0, 1.0, 5.0], [4.0, 0.0, 5.0]])
    acc, cnt = DS.accumulate(acc, cnt, g, np.array([1, 2, 0]), sx=2.0, sy=0.5)
    np.testing.assert_allclose(acc, [math.hypot(6.0, 2.0), 2.0, 0.0])
    assert cnt.tolist() == [1.0, 1.0, 0.0]


@pytest.mark.parametrize("o", [0.01, 0.3, 0.5, 0.9, 0.999])
def test_two_coincident_clones_composite_like_their_parent_at_its_centre(o):
    """The clone's opacity rule against the plain compositor: one splat of opacity o, and two coincident copies of
    opacity sigmoid(clone_logit(logit o)); equal at the pixel where the Gaussian factor is 1, close around it."""
    from oracle import composite as OC
    x = math.log(o / (1.0 - o))
    o2 = 1.0 / (1.0 + math.exp(-DS.clone_logit(x)))
    W, H = 21, 21
    one = {"xy": np.array([[10.5, 10.5]]), "conic": np.array([[0.08, 0.01, 0.05]]), "opacity": np.array([o]),
           "rgb": np.array([[0.9, 0.4, 0.2]]), "depth": np.array([2.0])}
    two = {k: np.repeat(v, 2, 0) for k, v in one.items()}
    two["opacity"] = np.array([o2, o2])
    a = OC.composite_image(one, W, H, (0.1, 0.2, 0.3), alpha_min=0.0, alpha_max=1.0, t_min=0.0)
    b = OC.composite_image(two, W, H, (0.1, 0.2, 0.3), alpha_min=0.0, alpha_max=1.0, t_min=0.0)
    assert abs(a["t_final"][10, 10] - b["t_final"][10, 10]) < 1e-12
    assert np.abs(a["image"][:, 10, 10] - b["image"][:, 10, 10]).max() < 1e-12
    # off centre the pair is slightly more opaque: 1 - (1 - o'e)^2 - o e = o'^2 e (1 - e) >= 0
    assert (b["t_final"] <= a["t_final"] + 1e-15).all()
    assert np.abs(a["image"] - b["image"]).max() < 0.26 * o2 ** 2 + 1e-12
