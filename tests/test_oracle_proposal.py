"""Pins of the residual-proposal oracle (CPU)."""
import numpy as np
import torch

from oracle import proposal as OPr


def _weights(rng, scale=0.3):
    return dict(W1=rng.normal(0, scale, (64, 24)), b1=rng.normal(0, 0.1, 64), W2=rng.normal(0, scale, (64, 64)),
                b2=rng.normal(0, 0.1, 64), W3=rng.normal(0, scale, (12, 64)), b3=rng.normal(0, 0.1, 12))


def _stats(rng):
    return dict(in_mean=rng.normal(0, 1, 24), in_rstd=rng.uniform(0.5, 2.0, 24), out_mean=rng.normal(0, 1, 12),
                out_std=rng.uniform(0.5, 2.0, 12))


def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-30, 100), rng.normal(0, 1e30, 100),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-45]])
    # exact ties: float32 values whose low 16 bits are 0x8000, with both parities of bit 16
    ties = (np.arange(1000, dtype=np.uint32) << 17 | 0x3F800000 | 0x8000).view(np.float32).astype(np.float64)
    ties2 = ((np.arange(1000, dtype=np.uint32) << 17) | (1 << 16) | 0x3F800000 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, ties2.astype(np.float64)])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = OPr.bf16_round(x)
    assert np.array_equal(got, ref)
    assert np.array_equal(np.signbit(got), np.signbit(ref))


def test_unrounded_forward_matches_torch_layers():
    rng = np.random.default_rng(1)
    W, st = _weights(rng), _stats(rng)
    x = rng.normal(0, 2, (24, 50))
    f = OPr.forward(x, W, st, rounding=False)
    F = torch.nn.functional
    xt = torch.tensor(x.T)
    xs = (xt - torch.tensor(st["in_mean"])) * torch.tensor(st["in_rstd"])
    h = F.silu(F.linear(xs, torch.tensor(W["W1"]), torch.tensor(W["b1"])))
    h = F.silu(F.linear(h, torch.tensor(W["W2"]), torch.tensor(W["b2"])))
    y = F.linear(h, torch.tensor(W["W3"]), torch.tensor(W["b3"])) * torch.tensor(st["out_std"]) + \
        torch.tensor(st["out_mean"])
    np.testing.assert_allclose(f["y"], y.numpy().T, rtol=1e-12, atol=1e-12)


def test_unrounded_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    W, st = _weights(rng), _stats(rng)
    x = rng.normal(0, 2, (24, 7))
    t = rng.normal(0, 1.5, (12, 7))
    _, g, _ = OPr.loss_and_grads(x, t, W, st, rounding=False)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = W[name].reshape(-1)
        for k in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[k]
            flat[k] = old + h
            lp, _, _ = OPr.loss_and_grads(x, t, W, st, rounding=False)
            flat[k] = old - h
            lm, _, _ = OPr.loss_and_grads(x, t, W, st, rounding=False)
            flat[k] = old
            fd = (lp - lm) / (2 * h)
            assert abs(g[name].reshape(-1)[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (name, k, g[name].reshape(-1)[k], fd)


def test_rounded_path_stays_within_bf16_error_of_the_unrounded_one():
    rng = np.random.default_rng(3)
    W, st = _weights(rng), _stats(rng)
    x = rng.normal(0, 2, (24, 200))
    t = rng.normal(0, 1.5, (12, 200))
    a = OPr.forward(x, W, st, rounding=True)["y"]
    b = OPr.forward(x, W, st, rounding=False)["y"]
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 2e-2
    _, ga, _ = OPr.loss_and_grads(x, t, W, st, rounding=True)
    _, gb, _ = OPr.loss_and_grads(x, t, W, st, rounding=False)
    for k in ga:
        assert np.linalg.norm(ga[k] - gb[k]) / np.linalg.norm(gb[k]) < 5e-2, k
    # operands really are bfloat16 values
    f = OPr.forward(x, W, st, rounding=True)
    for k in ("xb", "h1b", "h2b", "W1b"):
        v = f[k].astype(np.float32).view(np.uint32)
        assert np.all(v & 0xFFFF == 0), k


def test_features_hand_example():
    # two Gaussians; planes 0..9 of A_{t-1}, A_{t-2}, A_{t-3} chosen by hand, the other planes ignored
    A3 = np.zeros((59, 2))
    A2 = np.zeros((59, 2))
    A1 = np.zeros((59, 2))
    A3[0:10, 0] = np.arange(10)
    A2[0:10, 0] = np.arange(10) + 1.0
    A1[0:10, 0] = np.arange(10) + 3.0
    A1[20:, :] = 99.0  # not read
    A1[0:3, 1] = [5.0, 6.0, 7.0]
    A2[0:3, 1] = [5.0, 6.0, 7.0]
    A3[0:3, 1] = [4.0, 6.0, 7.0]
    f = OPr.features(A1, A2, A3, [0.25, 0.75])
    assert f.shape == (24, 2)
    np.testing.assert_array_equal(f[0:3, 0], [3.0, 4.0, 5.0])
    np.testing.assert_array_equal(f[3:13, 0], np.full(10, 2.0))
    np.testing.assert_array_equal(f[13:23, 0], np.full(10, 1.0))
    np.testing.assert_array_equal(f[0:3, 1], [5.0, 6.0, 7.0])
    np.testing.assert_array_equal(f[3:13, 1], np.zeros(10))
    np.testing.assert_array_equal(f[13:16, 1], [1.0, 0.0, 0.0])
    np.testing.assert_array_equal(f[23], [0.25, 0.75])
