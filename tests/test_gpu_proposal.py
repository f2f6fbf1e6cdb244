"""Residual-proposal kernels against the oracle (GPU, through the C ABI).

Outputs and gradients within 1e-3 relative L2 of the FP64 oracle evaluated on the same bf16-rounded
operands (the kernels accumulate in FP32; an operand whose float32 value sits at a bf16 rounding tie may
round the other way, which stays far inside the bound); features bit-exact against float32 arithmetic.
"""
import numpy as np
import pytest
import torch

from _helpers import rel_l2, to_dev
from oracle import proposal as OPr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    from paper_2412_04469_amd import proposal, qg
    qg.lib()
    return qg, proposal


def _case(rng, n, scale=0.25):
    from paper_2412_04469_amd import proposal as P
    params = P.init_params(int(rng.integers(1 << 30))).astype(np.float64)
    params += rng.normal(0, 0.05, params.shape)  # non-zero biases too
    params = params.astype(np.float32)
    stats = np.concatenate([rng.normal(0, 1, 24), rng.uniform(0.3, 3, 24), rng.normal(0, 1, 12),
                            rng.uniform(0.3, 3, 12)]).astype(np.float32)
    x = (rng.normal(0, 1.5, (24, n)) * rng.uniform(0.2, 3, (24, 1))).astype(np.float32)
    t = rng.normal(0, 2, (12, n)).astype(np.float32)
    return params, stats, x, t


def _oracle_args(P, params, stats):
    W = {k: v.astype(np.float64) for k, v in P.unpack(params).items()}
    st = dict(in_mean=stats[0:24].astype(np.float64), in_rstd=stats[24:48].astype(np.float64),
              out_mean=stats[48:60].astype(np.float64), out_std=stats[60:72].astype(np.float64))
    return W, st


@pytest.mark.parametrize("n", [1, 37, 1000, 70001])
def test_proposal_forward_parity(mods, n):
    qg, P = mods
    rng = np.random.default_rng(n)
    params, stats, x, _ = _case(rng, n)
    ld_in, ld_out = n + 5, n + 3  # padded leading dimensions
    X = torch.zeros(24, ld_in, device="cuda")
    X[:, :n] = to_dev(x)
    out = torch.full((12, ld_out), 7.0, device="cuda")
    qg.qg_proposal_fwd(n, ld_in, X, to_dev(params), to_dev(stats), out, ld_out)
    torch.cuda.synchronize()
    W, st = _oracle_args(P, params, stats)
    ref = OPr.forward(x.astype(np.float64), W, st, rounding=True)["y"]
    got = out[:, :n].cpu().numpy()
    assert rel_l2(got, ref) <= 1e-3, rel_l2(got, ref)
    assert np.abs(got - ref).max() <= 2e-2 * (np.abs(ref).max() + 1)
    assert torch.all(out[:, n:] == 7.0)  # nothing written past n


@pytest.mark.parametrize("m,S,gather", [(777, 3000, True), (4096, 4096, False), (5, 40, True)])
def test_proposal_backward_parity(mods, m, S, gather):
    qg, P = mods
    rng = np.random.default_rng(m + S)
    params, stats, x, t = _case(rng, S)
    idx = rng.choice(S, size=m, replace=False).astype(np.uint32) if gather else None
    cols = idx.astype(np.int64) if gather else np.arange(m)
    grad = torch.full((qg.PROPOSAL_PARAMS,), 0.5, device="cuda")  # accumulates (+=)
    loss = torch.zeros(1, device="cuda")
    wsb = qg.qg_proposal_bwd_workspace_size()
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    d_idx = None if idx is None else torch.as_tensor(idx.view(np.int32)).cuda()
    qg.qg_proposal_bwd(m, d_idx, S, S, to_dev(x), to_dev(t), to_dev(params), to_dev(stats), grad, loss, ws, wsb)
    torch.cuda.synchronize()
    W, st = _oracle_args(P, params, stats)
    ref_loss, ref_g, _ = OPr.loss_and_grads(x[:, cols].astype(np.float64), t[:, cols].astype(np.float64), W, st,
                                            rounding=True)
    np.testing.assert_allclose(loss.item(), ref_loss, rtol=1e-4)
    g = P.unpack(grad.cpu().numpy() - 0.5)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert rel_l2(g[k], ref_g[k]) <= 1e-3, (k, rel_l2(g[k], ref_g[k]))


def test_proposal_backward_is_deterministic(mods):
    qg, P = mods
    rng = np.random.default_rng(9)
    params, stats, x, t = _case(rng, 20000)
    wsb = qg.qg_proposal_bwd_workspace_size()
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    outs = []
    for _ in range(2):
        grad = torch.zeros(qg.PROPOSAL_PARAMS, device="cuda")
        qg.qg_proposal_bwd(20000, None, 20000, 20000, to_dev(x), to_dev(t), to_dev(params), to_dev(stats), grad, None,
                           ws, wsb)
        outs.append(grad.clone())
    assert torch.equal(outs[0], outs[1])


def test_proposal_features_exact(mods):
    qg, P = mods
    rng = np.random.default_rng(4)
    n, ld = 1001, 1010
    A = [rng.normal(0, 2, (59, ld)).astype(np.float32) for _ in range(3)]
    p = rng.uniform(0, 1, ld).astype(np.float32)
    out = torch.zeros(24, n + 2, device="cuda")
    qg.qg_proposal_features(n, ld, to_dev(A[0]), to_dev(A[1]), to_dev(A[2]), to_dev(p), out, n + 2)
    torch.cuda.synchronize()
    got = out[:, :n].cpu().numpy()
    ref = OPr.features(A[0][:, :n], A[1][:, :n], A[2][:, :n], p[:n])
    # the kernel subtracts in float32: compare with float32 arithmetic bit for bit
    ref32 = np.concatenate([A[0][0:3, :n], A[0][0:10, :n] - A[1][0:10, :n], A[1][0:10, :n] - A[2][0:10, :n],
                            p[None, :n]])
    assert np.array_equal(got, ref32)
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-6)


def test_proposal_training_fits_a_teacher(mods):
    """Adam on the library's gradients recovers a smooth teacher map (loss falls by over 10x)."""
    qg, P = mods
    rng = np.random.default_rng(5)
    S = 60000
    x = rng.normal(0, 1, (24, S)).astype(np.float32)
    Wt = rng.normal(0, 0.3, (12, 24))
    t = (np.tanh(Wt @ x) + 0.1 * (Wt @ x)).astype(np.float32)
    prop = P.Proposal(seed=3, lr=3e-3)
    X, T = to_dev(x), to_dev(t)
    prop.set_stats(X, T)
    losses = prop.train(X, T, steps=300, batch=8192, log_every=50)
    assert losses[-1][1] < losses[0][1] / 10, losses
    pred = prop.predict(X).cpu().numpy()
    assert rel_l2(pred, t) < 0.2
