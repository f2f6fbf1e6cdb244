"""Streaming fit and learned-proposal pipeline on a small dynamic scene (GPU)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_stream_and_proposal_pipeline_small():
    from paper_2412_04469_amd import stream, synth
    from paper_2412_04469_amd.fit import FitConfig
    wl = synth.workload_dynamic(n=4000, n_views=4, width=96, height=72)
    seq = stream.Sequence(wl, FitConfig(), torch.device("cuda"))
    recs, hist = stream.run_plain(seq, 6, iters=50, check_every=25)
    assert [r["t"] for r in recs] == list(range(1, 7))
    assert all(np.isfinite(r["target"]) and r["sec"] > 0 for r in recs)
    assert all(hist["y"][t].shape == (12, 4000) for t in range(1, 7))
    # the reconstruction of a frame differs from the previous one only where the fit moved it
    assert not torch.equal(hist["A"][1], hist["A"][0])
    prop, losses, _ = stream.train_proposal(hist, [1, 2, 3], steps=60, batch=4096)
    assert losses[-1][1] < losses[0][1]
    judged = stream.judge(seq, hist, recs, prop, [4, 5, 6], iters=50, check_every=25)
    assert [j["t"] for j in judged] == [4, 5, 6]
    s = stream.summarize(recs, judged, [4, 5, 6])
    assert s["frames"] == [4, 6]
    jb = stream.judge(seq, hist, recs, prop, [4, 5], iters=50, check_every=25, batched=True)
    assert len(jb) == 2


def test_fitter_does_not_alias_its_initial_attributes():
    """reset_frame(prev_attrs=...) writes the fitter's own copy of A_{t-1}, never the tensor it was built from
    (a streaming history handed to a fitter must stay intact)."""
    import torch
    from paper_2412_04469_amd import synth
    from paper_2412_04469_amd.fit import FitConfig, FrameFitter, render_views
    wl = synth.workload_fit_local(n=2000, width=96, height=64, n_views=2, frac_move=0.05)
    cfg = FitConfig()
    A0 = torch.as_tensor(wl.scene.planes()).cuda()
    keep = A0.clone()
    gts = render_views(A0, wl.cams, cfg)
    f = FrameFitter(A0, wl.cams, gts, cfg)
    f.reset_frame(prev_attrs=torch.as_tensor(wl.target_scene.planes()).cuda())
    torch.cuda.synchronize()
    assert torch.equal(A0, keep)


def test_proposal_reaches_the_plain_target_in_fewer_iterations():
    """What the trained residual proposal gains, on the 50-frame dynamic workload's first 30 frames (300 k
    Gaussians, 10% on sinusoids, 20 views at 1352x1014): the network is trained on the plain fits of frames 1-25
    and judged on frames 26-30; proposal-initialised frames reach each frame's plain target PSNR (the plain fit's
    held-out PSNR after 500 iterations) in fewer optimiser iterations on average than the plain, zero-initialised
    fit.  Iterations are counted (not time), with the adjoints in deterministic mode so that the counts do not
    depend on the order of float atomics."""
    from paper_2412_04469_amd import qg, stream, synth
    from paper_2412_04469_amd.fit import FitConfig
    qg.qg_set_deterministic(True)
    try:
        wl = synth.workload_dynamic()
        seq = stream.Sequence(wl, FitConfig(), torch.device("cuda"))
        say = lambda m: print(m, flush=True)  # one line per frame
        recs, hist = stream.run_plain(seq, 30, iters=500, check_every=25, log=say)
        prop, losses, _ = stream.train_proposal(hist, list(range(1, 26)), log=say)
        assert losses[-1][1] < losses[0][1]
        judged = stream.judge(seq, hist, recs, prop, list(range(26, 31)), iters=500, check_every=25, log=say)
        s = stream.summarize(recs, judged, list(range(26, 31)))
        print("proposal:", s, flush=True)
        assert s["frames_reaching_target"] == 5
        assert s["frames_using_proposal"] >= 4
        assert s["mean_iters_to_target"] < s["plain_mean_iters_to_target"]
    finally:
        qg.qg_set_deterministic(False)
