"""The FP32 FMA probe used by the benchmark's measured ceiling (GPU): every thread's 16 chains
a <- 0.999 a + 1e-4, started at (tid + k) * 1e-3, summed.  Checked against the same recurrence in FP64 on the
host (each FMA rounds once in FP32, so the chains agree to a few ulps of their magnitude)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_fma_probe_matches_the_recurrence():
    from paper_2412_04469_amd import qg
    blocks, iters = 3, 50
    out = torch.full((blocks * 256,), float("nan"), device="cuda")
    qg.qg_probe_fma(blocks, iters, out)
    torch.cuda.synchronize()
    tid = np.arange(256, dtype=np.float64)
    a = np.stack([(tid + k).astype(np.float32).astype(np.float64) * np.float64(np.float32(1e-3)) for k in range(16)])
    x, y = np.float64(np.float32(0.999)), np.float64(np.float32(1e-4))
    for _ in range(iters):
        a = a * x + y
    want = np.tile(a.sum(0), blocks)
    got = out.cpu().numpy().astype(np.float64)
    assert np.isfinite(got).all()
    np.testing.assert_allclose(got, want, rtol=1e-5)


def test_fma_probe_rejects_bad_arguments():
    from paper_2412_04469_amd import qg
    out = torch.empty(256, device="cuda")
    with pytest.raises(qg.QGError):
        qg.qg_probe_fma(0, 10, out)
    with pytest.raises(qg.QGError):
        qg.qg_probe_fma(1, 0, out)
