"""Host-side checks of the fit path, on the CPU with no kernel launched.

qg_bin never writes a negative pair count, so a negative one means a corrupt count buffer (and invalid tile
lists).  Every place that reads the pair count -- the rasterizer's capacity check, both fitters, the streaming
driver -- must turn it into a QGError instead of treating it as "no overflow".  The value is written into
num_pairs from the host."""
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


def test_rasterizer_pair_count_rejects_a_negative_count():
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
        assert e.value.status == qg.QG_ERR_HIP and "invalid pair count" in str(e.value)


def test_capacity_sizing_keeps_very_long_tile_lists_on_the_depth_passes():
    """fit_capacity sizes for the pair count (the per-tile route when that is at most 512 pairs per tile on
    average), unless a tile list is longer than the per-tile route sorts in LDS: then the capacity stays above
    512 per tile, where qg_bin takes the depth passes.  Ranges are written from the host."""
    from paper_2412_04469_amd import raster as R
    cams, _, _ = _setup(n=50, views=2)
    r = Rasterizer(50, cams, device="cpu", capacity=100)
    T = r.total_tiles
    r.ranges.zero_()
    r.ranges[0, 1] = 300
    assert r.longest_list() == 300
    assert r.fit_capacity(2000, 1.5, r.longest_list()) and r.capacity == 3000
    assert r.capacity <= R.PER_TILE_AVG * T
    r.ranges[1, 0], r.ranges[1, 1] = 300, 300 + R.PER_TILE_LIST_MAX + 1
    assert r.longest_list() == R.PER_TILE_LIST_MAX + 1
    assert r.fit_capacity(2000, 1.5, r.longest_list()) and r.capacity == R.PER_TILE_AVG * T + 1
    assert not r.fit_capacity(2000, 1.5, r.longest_list())  # already sized
    assert r.fit_capacity(2000, 1.5, 0) and r.capacity == 3000  # back on the per-tile route


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


def test_autotune_cache_returns_the_stored_choice(tmp_path):
    import json

    from paper_2412_04469_amd import autotune as AT
    cams, _, _ = _setup(n=10, views=3)
    key = AT.cache_key(cams, 500_000)
    assert key.endswith("|V3") and "n2^19" in key
    path = str(tmp_path / "tune.json")
    with open(path, "w") as f:
        json.dump({key: {"tile": [32, 8], "batch": 256, "heaviest_first": False, "ms": 6.1}}, f)

    def never(**_):
        raise AssertionError("a cached choice must not be timed")

    best, table = AT.autotune(never, cache_path=path, key=key)
    assert best == {"tile": (32, 8), "batch": 256, "heaviest_first": False} and table == []
    assert len(AT.candidates()) == 24


def test_grouping_tuner_picks_the_fastest_reaching_candidate():
    from paper_2412_04469_amd.autotune import tune_grouping
    secs = {(2, 1.5): None, (4, 2.5): 0.31, (5, 2.0): 0.29, (10, 3.0): 1.2}
    best, table = tune_grouping(lambda v, l: secs[(v, l)])
    assert best == (5, 2.0) and len(table) == 4
    assert tune_grouping(lambda v, l: None)[0] is None
