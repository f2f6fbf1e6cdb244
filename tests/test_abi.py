"""The C-ABI library loads, exports every entry point include/qg.h declares, and validates arguments
before touching the GPU (these calls return QG_ERR_ARG with nothing enqueued, so they run on the CPU)."""
import ctypes
import os
import re

import pytest

from paper_2412_04469_amd import qg, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(qg_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 18
    lib = ctypes.CDLL(qg.LIB_PATH)
    for nm in names:
        assert hasattr(lib, nm), nm
    assert qg.qg_version() == 2


def _cam(w=64, h=48):
    return synth.make_camera((0, 0, -4), w, h)


def test_bad_arguments_are_rejected_before_launch():
    with pytest.raises(qg.QGError) as e:
        qg.qg_project(10, 5, 1, 3, [_cam()], qg.tiling(16, 16), 0.3, [dict(splat=1, depth=1, rect=1, ntiles=1, flags=1)],
                      stream=0)
    assert e.value.status == qg.QG_ERR_ARG and "ld" in str(e.value)
    with pytest.raises(qg.QGError) as e:
        qg.qg_project(10, 10, 1, 4, [_cam()], qg.tiling(16, 16), 0.3, [dict(splat=1, depth=1, rect=1, ntiles=1, flags=1)],
                      stream=0)
    assert "sh_degree" in str(e.value)
    with pytest.raises(qg.QGError) as e:
        qg.qg_project(10, 10, 1, 3, [_cam()], qg.tiling(16, 8), 0.3, [dict(splat=1, depth=1, rect=1, ntiles=1, flags=1)],
                      stream=0)
    assert "tiling" in str(e.value)
    bad = _cam()
    bad.z_near = 0.0
    with pytest.raises(qg.QGError) as e:
        qg.qg_project(10, 10, 1, 3, [bad], qg.tiling(16, 16), 0.3, [dict(splat=1, depth=1, rect=1, ntiles=1, flags=1)],
                      stream=0)
    assert "z_near" in str(e.value)
    with pytest.raises(qg.QGError) as e:
        qg.qg_bin(10, [dict(splat=1, depth=1, rect=1, ntiles=1, flags=1)], [_cam()], qg.tiling(16, 16), 100, 1, None,
                  1, 1, 1, 10, stream=0)
    assert "workspace" in str(e.value)
    with pytest.raises(qg.QGError) as e:
        qg.qg_decode_residuals(10, 10, 1, 1, 8, 1, 1, 32, 56, 1, 1, 0.5, 1.01, 0.3, 2, stream=0)
    assert "gamma" in str(e.value)
    with pytest.raises(qg.QGError) as e:
        qg.qg_decode_residuals(10, 10, 1, 1, 4, 1, 1, 32, 56, 1, 1, -0.5, 1.01, 0.3, 2, stream=0)
    assert e.value.status == qg.QG_ERR_UNSUPPORTED
    with pytest.raises(qg.QGError):
        qg.qg_adam(10, 1, 1, 1, 1, 0.1, 0.9, 0.999, 1e-8, 0, stream=0)
    seg = (qg.qg_adam_segment * 9)()
    with pytest.raises(qg.QGError) as e:
        qg.qg_adam_multi(seg, 0.9, 0.999, 1e-8, 1, stream=0)
    assert "nseg" in str(e.value)
    seg = (qg.qg_adam_segment * 1)()
    seg[0] = qg.qg_adam_segment(None, None, None, None, 5, 0.1)
    with pytest.raises(qg.QGError) as e:
        qg.qg_adam_multi(seg, 0.9, 0.999, 1e-8, 1, stream=0)
    assert "NULL" in str(e.value)
    # the fused adjoint needs the attributes from somewhere: prev_attrs or the forward's decoded attributes
    P = dict(splat=1, depth=1, rect=1, ntiles=1, flags=1)
    ws = qg.qg_render_decode_bwd_workspace_size(10, 1)
    with pytest.raises(qg.QGError) as e:
        qg.qg_render_decode_bwd(10, 10, None, 1, 8, 1, 1, 32, 56, 1, 1, -0.5, 1.01, 0.3, 0.01, 3, [_cam()],
                                qg.tiling(16, 16), 0.3, [P], 1, 1, (0, 0, 0), [1], [1], [1], 1, 1, 1, 1, 1, None, None,
                                1, ws, stream=0, attrs=None)
    assert e.value.status == qg.QG_ERR_ARG and "NULL" in str(e.value)
    with pytest.raises(qg.QGError) as e:  # a workspace smaller than the query is refused
        qg.qg_render_decode_bwd(10, 10, None, 1, 8, 1, 1, 32, 56, 1, 1, -0.5, 1.01, 0.3, 0.01, 3, [_cam()],
                                qg.tiling(16, 16), 0.3, [P], 1, 1, (0, 0, 0), [1], [1], [1], 1, 1, 1, 1, 1, None, None,
                                1, ws - 1, stream=0, attrs=1)
    assert "workspace" in str(e.value)
    views = [_cam() for _ in range(17)]
    assert qg.qg_total_tiles(views, qg.tiling(16, 16)) == -1
    assert qg.qg_total_tiles([_cam(100, 70)], qg.tiling(32, 8)) == 4 * 9


def _rejects(call, *words, status=None):
    with pytest.raises(qg.QGError) as e:
        call()
    assert e.value.status == (qg.QG_ERR_ARG if status is None else status), str(e.value)
    for w in words:
        assert w in str(e.value), (w, str(e.value))


def test_mask_ssim_and_symbol_calls_reject_bad_arguments_before_launch():
    # D-SSIM: sizes, outputs, workspace, and the 2^31-pixel plane limit of its 32-bit staging offsets
    ws = qg.qg_ssim_workspace_size(3, 40, 50)
    _rejects(lambda: qg.qg_ssim_loss(0, 40, 50, 1, 1, 0.2, 1, 1, 1, ws, stream=0), "C=0")
    _rejects(lambda: qg.qg_ssim_loss(3, 40, 50, None, 1, 0.2, 1, 1, 1, ws, stream=0), "NULL")
    _rejects(lambda: qg.qg_ssim_loss(3, 40, 50, 1, 1, 0.2, None, None, 1, ws, stream=0), "nothing to compute")
    _rejects(lambda: qg.qg_ssim_loss(3, 40, 50, 1, 1, 0.2, 1, 1, 1, ws - 1, stream=0), "workspace")
    big = qg.qg_ssim_workspace_size(1, 1 << 16, 1 << 15)
    _rejects(lambda: qg.qg_ssim_loss(1, 1 << 16, 1 << 15, 1, 1, 0.2, 1, 1, 1, big, stream=0), "too large")
    assert qg.qg_ssim_workspace_size(0, 1, 1) == 0
    # masked L1: whole planes, 32-bit pixel count
    _rejects(lambda: qg.qg_l1_loss_masked(10, 3, 1, 1, 1, 1.0, 1, 1, stream=0), "multiple")
    _rejects(lambda: qg.qg_l1_loss_masked(3 << 32, 3, 1, 1, 1, 1.0, 1, 1, stream=0), "2^32")
    _rejects(lambda: qg.qg_l1_loss_masked(12, 3, 1, 1, None, 1.0, 1, 1, stream=0), "NULL")
    # the dynamic split, dilation and tile ranges of masked training
    _rejects(lambda: qg.qg_dynamic_flags(10, 1, 0.0, 1.0, 1e-3, 1, stream=0), "sx")
    _rejects(lambda: qg.qg_dynamic_flags(10, 1, 1.0, 1.0, -1.0, 1, stream=0), "t_d")
    _rejects(lambda: qg.qg_dilate_mask([_cam()], qg.tiling(16, 16), 0, [1], [1], [1], 1, stream=0), "k=0")
    _rejects(lambda: qg.qg_dilate_mask([_cam()], qg.tiling(16, 16), 48, [1], [None], [1], 1, stream=0), "NULL")
    _rejects(lambda: qg.qg_mask_tile_ranges(0, 1, 1, stream=0), "total_tiles")
    # latent symbols: L in [1, 16], ld >= n
    _rejects(lambda: qg.qg_latent_symbols(10, 10, 1, 17, 1, 1, 1, stream=0), "L=17")
    _rejects(lambda: qg.qg_latent_symbols(10, 5, 1, 8, 1, 1, 1, stream=0), "ld=5")


def test_workspace_queries():
    assert qg.qg_bin_workspace_size(1000, 2, 50000, 100) > 0
    assert qg.qg_render_bwd_workspace_size(1000, 3) >= 3 * 1000 * 12 * 4
    assert qg.qg_decode_bwd_workspace_size(1000, 8, 32, 56) > 0
    assert qg.qg_decode_lreg_blocks(257) == 2
