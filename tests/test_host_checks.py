"""Host-side checks of the fit path, on the CPU with no kernel launched.

A binning whose sort gave up waiting reports num_pairs = -1 (its tile lists are invalid).  Every place that
reads the pair count -- the rasterizer's capacity check, both fitters, the streaming driver -- must turn that
into a QGError instead of treating it as "no overflow".  The value is written into num_pairs from the host."""
import numpy as np
import pytest
import torch

from paper_2412_04469_amd import qg, synth
from paper_2412_04469_amd import stream as S
from paper_2412_04469_amd.fit import BatchedFitter, FitConfig, FrameFitter
from paper_2412_04469_amd.raster import Rasterizer


def _setup(n=50, views=2):
    cams = [synth.make_camera((0.3 * v, 0.0, -4.0), 48, 32) for v in range(views)]
    sc = synth.draw_scene(synth.rng_for(5), n)
    prev = torch.as_tensor(sc.planes())
    gts = [torch.zeros(3, 32, 48) for _ in cams]
    return cams, prev, gts


def test_rasterizer_pair_count_rejects_a_failed_sort():
    cams, prev, _ = _setup()
    r = Rasterizer(50, cams, device="cpu", capacity=100)
    r.num_pairs[0] = 40
    assert r.pair_count() == 40 and not r.overflowed() and not r.ensure_capacity()
    r.num_pairs[0] = 150
    assert r.overflowed()
    r.num_pairs[0] = -1
    for call in (r.pair_count, r.overflowed, r.ensure_capacity):
        with pytest.raises(qg.QGError) as e:
            call()
        assert e.value.status == qg.QG_ERR_HIP and "sort failure" in str(e.value)


def test_fitters_and_stream_reject_a_failed_sort():
    cams, prev, gts = _setup()
    bf = BatchedFitter(prev, cams, gts, FitConfig(), graph=False)
    bf.rasts[0].num_pairs[0] = 10
    assert not bf.overflowed()
    bf.rasts[0].num_pairs[0] = -1
    with pytest.raises(qg.QGError):
        bf.overflowed()
    with pytest.raises(qg.QGError):
        S._check_capacity(bf)
    ff = FrameFitter(prev, cams, gts, FitConfig())
    ff.rast.num_pairs[0] = -1
    with pytest.raises(qg.QGError):
        S._check_capacity(ff)
    ff.rast.num_pairs[0] = ff.rast.capacity + 5000  # a true overflow grows the buffers instead
    want = ff.rast.capacity + 5000
    assert S._check_capacity(ff) and ff.rast.capacity >= want


def test_attribute_fitter_builds_its_tables_on_the_host():
    from paper_2412_04469_amd.fit import AttributeFitter
    cams, prev, gts = _setup(n=40, views=2)
    f = AttributeFitter(prev, cams, gts, FitConfig(), graph=False)
    assert len(f.adam_segs) == 5
    ld = prev.shape[1]
    assert [f.adam_segs[k].count for k in range(5)] == [3 * ld, 4 * ld, 3 * ld, ld, 48 * ld]
    f.rast.num_pairs[0] = -1
    with pytest.raises(qg.QGError):
        f.overflowed()
