"""Thin ctypes binding of ``libqg.so`` (the C ABI in ``include/qg.h``), argument marshalling only.

Every function has the name of its C entry point.  Device buffers are passed as torch tensors (or raw
integer addresses); host structures (cameras, tiling, projected-buffer tables) are built here.  A
non-OK status raises ``QGError`` with ``qg_last_error()``.  Loading fails loudly if the library has
not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqg.so")

QG_OK = 0
QG_ERR_ARG = -1
QG_ERR_HIP = -2
QG_ERR_UNSUPPORTED = -3
N_PLANES = 59
MAX_VIEWS = 16
SPLAT_STRIDE = 12


class QGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"qg status {status}: {msg}")
        self.status = status


class qg_camera(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("z_near", ctypes.c_float)]


class qg_tiling(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("schedule", ctypes.c_void_p)]


class qg_adam_segment(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("m", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("count", ctypes.c_int64), ("lr", ctypes.c_float)]


class qg_projected(ctypes.Structure):
    _fields_ = [("splat", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("rect", ctypes.c_void_p),
                ("ntiles", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2412_04469_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32, f32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_size_t
        CAM = ctypes.POINTER(qg_camera)
        PRJ = ctypes.POINTER(qg_projected)
        sig = {
            "qg_last_error": ([], ctypes.c_char_p),
            "qg_version": ([], i32),
            "qg_set_deterministic": ([i32], i32),
            "qg_get_deterministic": ([], i32),
            "qg_deterministic_workspace_size": ([i64, i32, i64], sz),
            "qg_zero": ([P, i64, P], i32),
            "qg_probe_fma": ([i32, i32, P, P], i32),
            "qg_total_tiles": ([CAM, i32, qg_tiling], i64),
            "qg_decode_residuals": ([i64, i64, P, P, i32, P, P, i32, i32, P, P, P, f32, f32, f32, P, P, P, P], i32),
            "qg_decode_lreg_blocks": ([i64], i64),
            "qg_decode_lreg_mean": ([i64, P, i64, P, P], i32),
            "qg_decode_lreg_bwd": ([i64, P, f32, f32, f32, P, P, P], i32),
            "qg_decode_bwd_workspace_size": ([i64, i32, i32, i32], sz),
            "qg_decode_residuals_bwd": ([i64, i64, P, i32, P, P, i32, i32, P, P, P, f32, f32, f32, P, f32, P, P, P, P,
                                         P, P, sz, P], i32),
            "qg_project": ([i64, i64, P, i32, CAM, i32, qg_tiling, f32, PRJ, P], i32),
            "qg_bin_workspace_size": ([i64, i32, i64, i64], sz),
            "qg_bin": ([i64, PRJ, CAM, i32, qg_tiling, i64, P, P, P, P, P, sz, P], i32),
            "qg_bin_noalloc": ([i64, PRJ, CAM, i32, qg_tiling, i64, P, P, P, P, P], i32),
            "qg_bin_noalloc_max_bytes": ([], sz),
            "qg_render_fwd": ([PRJ, CAM, i32, qg_tiling, P, P, P, P, P, P, P], i32),
            "qg_render_fwd_l1": ([PRJ, CAM, i32, qg_tiling, P, P, P, P, P, P, P, P, P, P, P], i32),
            "qg_render_bwd_workspace_size": ([i64, i32], sz),
            "qg_render_bwd": ([i64, i64, P, i32, CAM, i32, qg_tiling, f32, PRJ, P, P, P, P, P, P, P, P, P, P, sz, P],
                              i32),
            "qg_loss_blocks": ([i64], i64),
            "qg_l1_loss": ([i64, P, P, f32, P, P, P], i32),
            "qg_l1_loss_masked": ([i64, i64, P, P, P, f32, P, P, P], i32),
            "qg_ssim_workspace_size": ([i32, i32, i32], sz),
            "qg_latent_symbols": ([i64, i64, P, i32, P, P, P, P], i32),
            "qg_rans_bound": ([i64], sz),
            "qg_rans_encode": ([i64, i32, P, P, P, sz, ctypes.POINTER(ctypes.c_size_t)], i32),
            "qg_rans_decode": ([i64, i32, P, sz, P, P], i32),
            "qg_ssim_loss": ([i32, i32, i32, P, P, f32, P, P, P, sz, P], i32),
            "qg_dynamic_flags": ([i64, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P], i32),
            "qg_dynamic_mask": ([PRJ, CAM, i32, qg_tiling, P, P, P, P, P], i32),
            "qg_dilate_mask": ([CAM, i32, qg_tiling, i32, P, P, P, P, P], i32),
            "qg_mask_tile_ranges": ([i64, P, P, P], i32),
            "qg_loss_reduce": ([i64, P, P, P], i32),
            "qg_loss_reduce_parts": ([i64, i64, P, P, P], i32),
            "qg_adam": ([i64, P, P, P, P, f32, f32, f32, f32, i32, P], i32),
            "qg_timing_enable": ([i32, ctypes.c_char_p], i32),
            "qg_adam_multi": ([i32, ctypes.POINTER(qg_adam_segment), f32, f32, f32, i32, P, i32, P], i32),
            "qg_decode_project_lreg_blocks": ([i64], i64),
            "qg_scaled_diff": ([i64, P, P, f32, P, P], i32),
            "qg_gate_init_workspace_size": ([i64], sz),
            "qg_gate_init": ([i64, P, f32, f32, f32, P, P, P, P, sz, P], i32),
            "qg_decode_project": ([i64, i64, P, P, i32, P, P, i32, i32, P, P, P, f32, f32, f32, i32, CAM, i32,
                                   qg_tiling, f32, PRJ, P, P, P, P], i32),
            "qg_render_decode_bwd_workspace_size": ([i64, i32], sz),
            "qg_render_decode_bwd": ([i64, i64, P, P, P, i32, P, P, i32, i32, P, P, P, f32, f32, f32, f32, i32, CAM,
                                      i32, qg_tiling, f32, PRJ, P, P, P, P, P, P, P, P, P, P, P, P, P, P, sz, P], i32),
            "qg_timing_report": ([ctypes.c_char_p, i64], i64),
            "qg_schedule_words": ([i64], i64),
            "qg_proposal_features": ([i64, i64, P, P, P, P, P, i64, P], i32),
            "qg_proposal_fwd": ([i64, i64, P, P, P, P, i64, P], i32),
            "qg_proposal_bwd_workspace_size": ([], sz),
            "qg_proposal_bwd": ([i64, P, i64, i64, P, P, P, P, P, P, P, sz, P], i32),
            "qg_schedule_tiles": ([CAM, i32, qg_tiling, P, P, i64, P], i32),
            "qg_gate_noise": ([i64, ctypes.c_uint64, i32, P, P, P], i32),
            "qg_linear_decoder_params": ([ctypes.POINTER(i32)], i64),
            "qg_decode_linear_blocks": ([i64], i64),
            "qg_decode_linear": ([i64, i64, P, P, ctypes.POINTER(i32), P, P, P, P, f32, f32, f32, P, P, P, P], i32),
            "qg_decode_linear_bwd_workspace_size": ([i64, ctypes.POINTER(i32)], sz),
            "qg_decode_linear_bwd": ([i64, i64, P, ctypes.POINTER(i32), P, P, P, P, f32, f32, f32, P, f32, P, P, P, P,
                                      P, sz, P], i32),
            "qg_densify_accumulate": ([i64, P, P, f32, f32, P, P, P], i32),
            "qg_densify_plan_workspace_size": ([i64], sz),
            "qg_densify_plan": ([i64, P, P, P, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P, P, sz,
                                 P], i32),
            "qg_densify_expand": ([i64, P, P, i32, P, i64, P, i64, i32, P], i32),
            "qg_densify_children": ([i64, P, P, P, i64, ctypes.c_uint64, i32, P, i64, P], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return [n for n in dir(lib()) if n.startswith("qg_")]


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(status):
    if status != QG_OK:
        raise QGError(status, lib().qg_last_error().decode())


def make_camera(cam) -> qg_camera:
    """qg_camera from an object with fx, fy, cx, cy, R [3,3], t [3], width, height, z_near."""
    c = qg_camera()
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, np.float32).reshape(9)
    t = np.asarray(cam.t, np.float32).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.width, c.height, c.z_near = int(cam.width), int(cam.height), float(cam.z_near)
    return c


def camera_array(cams):
    if isinstance(cams, ctypes.Array):
        return cams
    arr = (qg_camera * len(cams))()
    for k, c in enumerate(cams):
        arr[k] = c if isinstance(c, qg_camera) else make_camera(c)
    return arr


def tiling(tw=16, th=16, batch=0, schedule=None) -> qg_tiling:
    """Tile shape, blend batch depth (0 = 64) and optional heaviest-first schedule buffer (device tensor)."""
    return qg_tiling(int(tw), int(th), int(batch), 0, _ptr(schedule))


def projected_array(bufs):
    """bufs: list of dicts with splat, depth, rect, ntiles, flags tensors."""
    if isinstance(bufs, ctypes.Array):
        return bufs
    arr = (qg_projected * len(bufs))()
    for k, b in enumerate(bufs):
        arr[k] = qg_projected(_ptr(b["splat"]), _ptr(b["depth"]), _ptr(b["rect"]), _ptr(b["ntiles"]), _ptr(b["flags"]))
    return arr


def _ptr_array(xs):
    if isinstance(xs, ctypes.Array):
        return xs
    arr = (ctypes.c_void_p * len(xs))()
    for k, x in enumerate(xs):
        arr[k] = _ptr(x)
    return arr


# ---------------------------------------------------------------------------------------------- calls

def qg_version():
    return lib().qg_version()


def qg_zero(dst, nbytes, stream=None):
    _check(lib().qg_zero(_ptr(dst), int(nbytes), _stream(stream)))


def qg_probe_fma(blocks, iters, out, stream=None):
    _check(lib().qg_probe_fma(int(blocks), int(iters), _ptr(out), _stream(stream)))


PROPOSAL_PARAMS = 6540


def qg_proposal_features(n, ld, A1, A2, A3, p, out, ld_out, stream=None):
    _check(lib().qg_proposal_features(int(n), int(ld), _ptr(A1), _ptr(A2), _ptr(A3), _ptr(p), _ptr(out), int(ld_out),
                                      _stream(stream)))


def qg_proposal_fwd(n, ld_in, features, params, stats, out, ld_out, stream=None):
    _check(lib().qg_proposal_fwd(int(n), int(ld_in), _ptr(features), _ptr(params), _ptr(stats), _ptr(out),
                                 int(ld_out), _stream(stream)))


def qg_proposal_bwd_workspace_size():
    return int(lib().qg_proposal_bwd_workspace_size())


def qg_proposal_bwd(m, idx, n, ld, features, targets, params, stats, grad, loss_out, ws, ws_bytes, stream=None):
    _check(lib().qg_proposal_bwd(int(m), _ptr(idx), int(n), int(ld), _ptr(features), _ptr(targets), _ptr(params),
                                 _ptr(stats), _ptr(grad), _ptr(loss_out), _ptr(ws), int(ws_bytes), _stream(stream)))


def qg_schedule_words(total_tiles):
    return int(lib().qg_schedule_words(int(total_tiles)))


def qg_schedule_tiles(cams, tile, tile_ranges, schedule, stream=None):
    """cams: a camera_array (or a list of cameras); tile: the binning's qg_tiling."""
    ca = camera_array(cams)
    _check(lib().qg_schedule_tiles(ca, len(ca), tile, _ptr(tile_ranges), _ptr(schedule), int(schedule.numel()),
                                   _stream(stream)))


def qg_total_tiles(cams, tile):
    ca = camera_array(cams)
    return int(lib().qg_total_tiles(ca, len(cams), tile))


def qg_decode_residuals(n, ld, prev_attrs, latents, L, W1, W2, Hd, M, pos_pre, gate_logit, gamma0, gamma1, tau,
                        attrs_out, gate_out=None, lreg_partial=None, stream=None, gate_noise=None):
    _check(lib().qg_decode_residuals(int(n), int(ld), _ptr(prev_attrs), _ptr(latents), int(L), _ptr(W1), _ptr(W2),
                                     int(Hd), int(M), _ptr(pos_pre), _ptr(gate_logit), _ptr(gate_noise),
                                     float(gamma0), float(gamma1),
                                     float(tau), _ptr(attrs_out), _ptr(gate_out), _ptr(lreg_partial),
                                     _stream(stream)))


def qg_decode_lreg_blocks(n):
    return int(lib().qg_decode_lreg_blocks(int(n)))


def qg_decode_lreg_mean(n, lreg_partial, nblocks, out, stream=None):
    _check(lib().qg_decode_lreg_mean(int(n), _ptr(lreg_partial), int(nblocks), _ptr(out), _stream(stream)))


def qg_decode_lreg_bwd(n, gate_logit, gamma0, gamma1, tau, weight, grad_gate_logit, stream=None):
    _check(lib().qg_decode_lreg_bwd(int(n), _ptr(gate_logit), float(gamma0), float(gamma1), float(tau), _ptr(weight),
                                    _ptr(grad_gate_logit), _stream(stream)))


def qg_decode_bwd_workspace_size(n, L, Hd, M):
    return int(lib().qg_decode_bwd_workspace_size(int(n), int(L), int(Hd), int(M)))


def qg_decode_residuals_bwd(n, ld, latents, L, W1, W2, Hd, M, pos_pre, gate_logit, gamma0, gamma1, tau, grad_attrs,
                            lambda_reg, grad_latents, grad_W1, grad_W2, grad_pos_pre, grad_gate_logit, ws, ws_bytes,
                            stream=None, gate_noise=None):
    _check(lib().qg_decode_residuals_bwd(int(n), int(ld), _ptr(latents), int(L), _ptr(W1), _ptr(W2), int(Hd), int(M),
                                         _ptr(pos_pre), _ptr(gate_logit), _ptr(gate_noise), float(gamma0),
                                         float(gamma1), float(tau),
                                         _ptr(grad_attrs), float(lambda_reg), _ptr(grad_latents), _ptr(grad_W1),
                                         _ptr(grad_W2), _ptr(grad_pos_pre), _ptr(grad_gate_logit), _ptr(ws),
                                         int(ws_bytes), _stream(stream)))


def qg_project(n, ld, attrs, sh_degree, cams, tile, dilation, out, stream=None):
    ca = camera_array(cams)
    pa = projected_array(out)
    _check(lib().qg_project(int(n), int(ld), _ptr(attrs), int(sh_degree), ca, len(cams), tile, float(dilation), pa,
                            _stream(stream)))


def qg_set_deterministic(on):
    _check(lib().qg_set_deterministic(1 if on else 0))


def qg_get_deterministic():
    return bool(lib().qg_get_deterministic())


def qg_deterministic_workspace_size(n, V, capacity):
    return int(lib().qg_deterministic_workspace_size(int(n), int(V), int(capacity)))


def qg_bin_workspace_size(n, V, capacity, total_tiles):
    return int(lib().qg_bin_workspace_size(int(n), int(V), int(capacity), int(total_tiles)))


def qg_bin(n, proj, cams, tile, capacity, vals, keys, tile_ranges, num_pairs, ws, ws_bytes, stream=None):
    ca = camera_array(cams)
    pa = projected_array(proj)
    _check(lib().qg_bin(int(n), pa, ca, len(cams), tile, int(capacity), _ptr(vals), _ptr(keys), _ptr(tile_ranges),
                        _ptr(num_pairs), _ptr(ws), int(ws_bytes), _stream(stream)))


def qg_bin_noalloc_max_bytes():
    return int(lib().qg_bin_noalloc_max_bytes())


def qg_bin_noalloc(n, proj, cams, tile, capacity, vals, keys, tile_ranges, num_pairs, stream=None):
    ca = camera_array(cams)
    pa = projected_array(proj)
    _check(lib().qg_bin_noalloc(int(n), pa, ca, len(cams), tile, int(capacity), _ptr(vals), _ptr(keys),
                                _ptr(tile_ranges), _ptr(num_pairs), _stream(stream)))


def qg_render_fwd(proj, cams, tile, vals, tile_ranges, bg, image, T_final, last, stream=None):
    ca = camera_array(cams)
    pa = projected_array(proj)
    bga = (ctypes.c_float * 3)(*[float(b) for b in bg])
    _check(lib().qg_render_fwd(pa, ca, len(cams), tile, _ptr(vals), _ptr(tile_ranges), bga, _ptr_array(image),
                               _ptr_array(T_final), _ptr_array(last), _stream(stream)))


def float_array(xs):
    """A [host] array of floats (e.g. the per-view scales of qg_render_fwd_l1)."""
    if isinstance(xs, ctypes.Array):
        return xs
    return (ctypes.c_float * len(xs))(*[float(x) for x in xs])


def qg_render_fwd_l1(proj, cams, tile, vals, tile_ranges, bg, image, T_final, last, gt, scale, grad_image, partials,
                     stream=None):
    ca = camera_array(cams)
    pa = projected_array(proj)
    bga = (ctypes.c_float * 3)(*[float(b) for b in bg])
    _check(lib().qg_render_fwd_l1(pa, ca, len(cams), tile, _ptr(vals), _ptr(tile_ranges), bga, _ptr_array(image),
                                  _ptr_array(T_final), _ptr_array(last), _ptr_array(gt), float_array(scale),
                                  _ptr_array(grad_image), _ptr(partials), _stream(stream)))


def qg_render_bwd_workspace_size(n, V):
    return int(lib().qg_render_bwd_workspace_size(int(n), int(V)))


def qg_render_bwd(n, ld, attrs, sh_degree, cams, tile, dilation, proj, vals, tile_ranges, bg, T_final, last,
                  grad_image, grad_attrs, grad_xy_abs, grad_xy, ws, ws_bytes, stream=None):
    ca = camera_array(cams)
    pa = projected_array(proj)
    bga = (ctypes.c_float * 3)(*[float(b) for b in bg])
    gxy = None if grad_xy is None else _ptr_array(grad_xy)
    _check(lib().qg_render_bwd(int(n), int(ld), _ptr(attrs), int(sh_degree), ca, len(cams), tile, float(dilation), pa,
                               _ptr(vals), _ptr(tile_ranges), bga, _ptr_array(T_final), _ptr_array(last),
                               _ptr_array(grad_image), _ptr(grad_attrs), _ptr(grad_xy_abs), gxy, _ptr(ws),
                               int(ws_bytes), _stream(stream)))


def qg_loss_blocks(count):
    return int(lib().qg_loss_blocks(int(count)))


def qg_l1_loss(count, image, gt, scale, grad_image, partials, stream=None):
    _check(lib().qg_l1_loss(int(count), _ptr(image), _ptr(gt), float(scale), _ptr(grad_image), _ptr(partials),
                            _stream(stream)))


def qg_l1_loss_masked(count, plane, image, gt, mask, scale, grad_image, partials, stream=None):
    _check(lib().qg_l1_loss_masked(int(count), int(plane), _ptr(image), _ptr(gt), _ptr(mask), float(scale),
                                   _ptr(grad_image), _ptr(partials), _stream(stream)))


def qg_latent_symbols(n, ld, latents, L, symbols, hist, overflow, stream=None):
    _check(lib().qg_latent_symbols(int(n), int(ld), _ptr(latents), int(L), _ptr(symbols), _ptr(hist), _ptr(overflow),
                                   _stream(stream)))


def _host(a):
    """Host pointer of a C-contiguous numpy array."""
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def qg_rans_encode(L, symbols, hist):
    """symbols: int8 numpy [count]; hist: uint32 numpy [L][256] -> coded bytes (numpy uint8)."""
    count = int(symbols.size)
    out = np.empty(int(lib().qg_rans_bound(count)), np.uint8)
    nb = ctypes.c_size_t(0)
    _check(lib().qg_rans_encode(count, int(L), _host(symbols), _host(hist), _host(out), out.size, ctypes.byref(nb)))
    return out[:nb.value].copy()


def qg_rans_decode(count, L, data, hist):
    out = np.empty(int(count), np.int8)
    _check(lib().qg_rans_decode(int(count), int(L), _host(data), int(data.size), _host(hist), _host(out)))
    return out


def qg_ssim_workspace_size(C, H, W):
    return int(lib().qg_ssim_workspace_size(int(C), int(H), int(W)))


def qg_ssim_loss(C, H, W, image, gt, weight, grad_image, dssim_out, ws, ws_bytes, stream=None):
    _check(lib().qg_ssim_loss(int(C), int(H), int(W), _ptr(image), _ptr(gt), float(weight), _ptr(grad_image),
                              _ptr(dssim_out), _ptr(ws), int(ws_bytes), _stream(stream)))


def qg_dynamic_flags(n, d, sx, sy, t_d, dynamic, stream=None):
    _check(lib().qg_dynamic_flags(int(n), _ptr(d), float(sx), float(sy), float(t_d), _ptr(dynamic), _stream(stream)))


def qg_dynamic_mask(proj, cams, tile, vals, tile_ranges, dynamic, mask, stream=None):
    ca = camera_array(cams)
    pa = projected_array(proj)
    _check(lib().qg_dynamic_mask(pa, ca, len(cams), tile, _ptr(vals), _ptr(tile_ranges), _ptr(dynamic),
                                 _ptr_array(mask), _stream(stream)))


def qg_dilate_mask(cams, tile, k, mask, tmp, dilated, tile_flags, stream=None):
    ca = camera_array(cams)
    _check(lib().qg_dilate_mask(ca, len(cams), tile, int(k), _ptr_array(mask), _ptr_array(tmp), _ptr_array(dilated),
                                _ptr(tile_flags), _stream(stream)))


def qg_mask_tile_ranges(total_tiles, tile_ranges, tile_flags, stream=None):
    _check(lib().qg_mask_tile_ranges(int(total_tiles), _ptr(tile_ranges), _ptr(tile_flags), _stream(stream)))


def qg_loss_reduce(count, partials, out, stream=None):
    _check(lib().qg_loss_reduce(int(count), _ptr(partials), _ptr(out), _stream(stream)))


def qg_loss_reduce_parts(nparts, count, partials, out, stream=None):
    _check(lib().qg_loss_reduce_parts(int(nparts), int(count), _ptr(partials), _ptr(out), _stream(stream)))


def qg_adam(count, param, grad, m, v, lr, b1, b2, eps, t, stream=None):
    _check(lib().qg_adam(int(count), _ptr(param), _ptr(grad), _ptr(m), _ptr(v), float(lr), float(b1), float(b2),
                         float(eps), int(t), _stream(stream)))


def qg_timing_enable(on, only=None):
    _check(lib().qg_timing_enable(int(bool(on)), None if only is None else only.encode()))


def qg_timing_report():
    """{name: (count, total_ms)} for the launches recorded since the last report (waits for them)."""
    buf = ctypes.create_string_buffer(1 << 16)
    lib().qg_timing_report(buf, len(buf))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


def qg_decode_project_lreg_blocks(n):
    return int(lib().qg_decode_project_lreg_blocks(int(n)))


def qg_decode_project(n, ld, prev_attrs, latents, L, W1, W2, Hd, M, pos_pre, gate_logit, gamma0, gamma1, tau,
                      sh_degree, cams, tile, dilation, out, attrs_out=None, gate_out=None, lreg_partial=None,
                      stream=None, gate_noise=None):
    ca = camera_array(cams)
    pa = projected_array(out)
    _check(lib().qg_decode_project(int(n), int(ld), _ptr(prev_attrs), _ptr(latents), int(L), _ptr(W1), _ptr(W2),
                                   int(Hd), int(M), _ptr(pos_pre), _ptr(gate_logit), _ptr(gate_noise),
                                   float(gamma0), float(gamma1),
                                   float(tau), int(sh_degree), ca, len(ca), tile, float(dilation), pa,
                                   _ptr(attrs_out), _ptr(gate_out), _ptr(lreg_partial), _stream(stream)))


def qg_render_decode_bwd_workspace_size(n, V):
    return int(lib().qg_render_decode_bwd_workspace_size(int(n), int(V)))


def qg_render_decode_bwd(n, ld, prev_attrs, latents, L, W1, W2, Hd, M, pos_pre, gate_logit, gamma0, gamma1, tau,
                         lambda_reg, sh_degree, cams, tile, dilation, proj, vals, tile_ranges, bg, T_final, last,
                         grad_image, grad_latents, grad_W1, grad_W2, grad_pos_pre, grad_gate_logit, grad_xy_abs,
                         grad_xy, ws, ws_bytes, stream=None, attrs=None, gate_noise=None):
    ca = camera_array(cams)
    pa = projected_array(proj)
    bga = (ctypes.c_float * 3)(*[float(b) for b in bg])
    gxy = None if grad_xy is None else _ptr_array(grad_xy)
    _check(lib().qg_render_decode_bwd(int(n), int(ld), _ptr(prev_attrs), _ptr(attrs), _ptr(latents), int(L), _ptr(W1),
                                      _ptr(W2),
                                      int(Hd), int(M), _ptr(pos_pre), _ptr(gate_logit), _ptr(gate_noise),
                                      float(gamma0), float(gamma1), float(tau), float(lambda_reg), int(sh_degree), ca,
                                      len(ca), tile,
                                      float(dilation), pa, _ptr(vals), _ptr(tile_ranges), bga, _ptr_array(T_final),
                                      _ptr_array(last), _ptr_array(grad_image), _ptr(grad_latents), _ptr(grad_W1),
                                      _ptr(grad_W2), _ptr(grad_pos_pre), _ptr(grad_gate_logit), _ptr(grad_xy_abs),
                                      gxy, _ptr(ws), int(ws_bytes), _stream(stream)))


def qg_scaled_diff(count, a, b, scale, out, stream=None):
    _check(lib().qg_scaled_diff(int(count), _ptr(a), _ptr(b), float(scale), _ptr(out), _stream(stream)))


def qg_gate_init_workspace_size(n):
    return int(lib().qg_gate_init_workspace_size(int(n)))


def qg_gate_init(n, d, gamma0, gamma1, tau, a_out, p_out, median_out, ws, ws_bytes, stream=None):
    _check(lib().qg_gate_init(int(n), _ptr(d), float(gamma0), float(gamma1), float(tau), _ptr(a_out), _ptr(p_out),
                              _ptr(median_out), _ptr(ws), int(ws_bytes), _stream(stream)))


def adam_segments(params, grads, ms, vs, lrs):
    """Host table for qg_adam_multi from parallel lists of tensors and learning rates."""
    arr = (qg_adam_segment * len(params))()
    for k, (p, g, m, v, lr) in enumerate(zip(params, grads, ms, vs, lrs)):
        arr[k] = qg_adam_segment(_ptr(p), _ptr(g), _ptr(m), _ptr(v), int(p.numel()), float(lr))
    return arr


def qg_adam_multi(segs, b1, b2, eps, t, zero_grad=True, stream=None, step_state=None):
    _check(lib().qg_adam_multi(len(segs), segs, float(b1), float(b2), float(eps), int(t), _ptr(step_state),
                               int(bool(zero_grad)), _stream(stream)))


def qg_gate_noise(n, seed, step, noise, step_state=None, stream=None):
    _check(lib().qg_gate_noise(int(n), int(seed) & 0xFFFFFFFFFFFFFFFF, int(step), _ptr(step_state), _ptr(noise),
                               _stream(stream)))


def qg_densify_accumulate(n, grad_xy, ntiles, sx, sy, accum, count, stream=None):
    _check(lib().qg_densify_accumulate(int(n), _ptr(grad_xy), _ptr(ntiles), float(sx), float(sy), _ptr(accum),
                                       _ptr(count), _stream(stream)))


def qg_densify_plan_workspace_size(n):
    return int(lib().qg_densify_plan_workspace_size(int(n)))


def qg_densify_plan(n, accum, count, attrs, ld, threshold, max_scale, min_opacity, action, offsets, ws, ws_bytes,
                    stream=None):
    _check(lib().qg_densify_plan(int(n), _ptr(accum), _ptr(count), _ptr(attrs), int(ld), float(threshold),
                                 float(max_scale), float(min_opacity), _ptr(action), _ptr(offsets), _ptr(ws),
                                 int(ws_bytes), _stream(stream)))


def qg_densify_expand(n, action, offsets, nplanes, src, ld_src, dst, ld_dst, mode, stream=None):
    _check(lib().qg_densify_expand(int(n), _ptr(action), _ptr(offsets), int(nplanes), _ptr(src), int(ld_src), _ptr(dst),
                                   int(ld_dst), int(mode), _stream(stream)))


def qg_densify_children(n, action, offsets, decoded, ld, seed, rnd, prev_out, ld_out, stream=None):
    _check(lib().qg_densify_children(int(n), _ptr(action), _ptr(offsets), _ptr(decoded), int(ld),
                                  int(seed) & 0xFFFFFFFFFFFFFFFF, int(rnd), _ptr(prev_out), int(ld_out),
                                  _stream(stream)))


def _dims(dims):
    return (ctypes.c_int32 * 5)(*[int(d) for d in dims])


def qg_linear_decoder_params(dims):
    return int(lib().qg_linear_decoder_params(_dims(dims)))


def qg_decode_linear_blocks(n):
    return int(lib().qg_decode_linear_blocks(int(n)))


def qg_decode_linear(n, ld, prev_attrs, latents, dims, D, pos_pre, gate_logit, gamma0, gamma1, tau, attrs_out,
                     gate_out=None, lreg_partial=None, stream=None, gate_noise=None):
    _check(lib().qg_decode_linear(int(n), int(ld), _ptr(prev_attrs), _ptr(latents), _dims(dims), _ptr(D), _ptr(pos_pre),
                                  _ptr(gate_logit), _ptr(gate_noise), float(gamma0), float(gamma1), float(tau),
                                  _ptr(attrs_out), _ptr(gate_out), _ptr(lreg_partial), _stream(stream)))


def qg_decode_linear_bwd_workspace_size(n, dims):
    return int(lib().qg_decode_linear_bwd_workspace_size(int(n), _dims(dims)))


def qg_decode_linear_bwd(n, ld, latents, dims, D, pos_pre, gate_logit, gamma0, gamma1, tau, grad_attrs, lambda_reg,
                         grad_latents, grad_D, grad_pos_pre, grad_gate_logit, ws, ws_bytes, stream=None,
                         gate_noise=None):
    _check(lib().qg_decode_linear_bwd(int(n), int(ld), _ptr(latents), _dims(dims), _ptr(D), _ptr(pos_pre),
                                      _ptr(gate_logit), _ptr(gate_noise), float(gamma0), float(gamma1), float(tau),
                                      _ptr(grad_attrs), float(lambda_reg), _ptr(grad_latents), _ptr(grad_D),
                                      _ptr(grad_pos_pre), _ptr(grad_gate_logit), _ptr(ws), int(ws_bytes),
                                      _stream(stream)))
