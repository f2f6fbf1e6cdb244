"""ctypes wrapper of the FP64 C compositor (``composite.c``); test infrastructure only.

Eq. 2 per pixel over all splats; see the C file header for the definition, the adjoint, and the
decision margins.  Pinned by: closed forms (single splat, footprint pixel count, termination count,
clamp), invariants (weights + T_final sum to 1, input-order invariance), the independent NumPy brute
force in ``brute.py``, central finite differences of its own forward, and agreement of the
stored-T and reverse-T adjoints.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "composite.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4


def build(force: bool = False) -> str:
    """Compile ``composite.c`` with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_composite.argtypes = [ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int64, P, P, P,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                         P, P, P, P, P, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_composite.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def composite(splats: dict, px: np.ndarray, py: np.ndarray, bg=(0.0, 0.0, 0.0), grad_color=None,
              alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX, t_min=T_MIN, reverse_t=False, nthreads=0):
    """Composite the given pixel centres.

    splats: dict with xy [N,2], conic [N,3], opacity [N], rgb [N,3], depth [N], optional valid [N] bool.
    Returns dict: color [M,3], t_final [M], last_id [M] (-1 if none), n_contrib [M], margin [M] (alpha and
    termination decisions), order_margin [M] (relative gap of adjacent depths) and, if
    ``grad_color`` [M,3] is given, g_xy [N,2], g_conic [N,3], g_opacity [N], g_rgb [N,3].
    """
    lib = _load()
    d = lambda k: np.ascontiguousarray(np.asarray(splats[k], np.float64))
    xy, conic, op, rgb, depth = d("xy"), d("conic"), d("opacity"), d("rgb"), d("depth")
    n = op.shape[0]
    valid = splats.get("valid")
    valid = None if valid is None else np.ascontiguousarray(np.asarray(valid, np.uint8))
    px = np.ascontiguousarray(np.asarray(px, np.float64))
    py = np.ascontiguousarray(np.asarray(py, np.float64))
    m = px.shape[0]
    bg = np.ascontiguousarray(np.asarray(bg, np.float64))
    color = np.zeros((m, 3))
    tf = np.zeros(m)
    last = np.zeros(m, np.int64)
    cnt = np.zeros(m, np.int32)
    margin = np.zeros(m)
    order = np.zeros(m)
    out = {"color": color, "t_final": tf, "last_id": last, "n_contrib": cnt, "margin": margin, "order_margin": order}
    g = [None] * 4
    gc = None
    if grad_color is not None:
        gc = np.ascontiguousarray(np.asarray(grad_color, np.float64).reshape(m, 3))
        g = [np.zeros((n, 2)), np.zeros((n, 3)), np.zeros(n), np.zeros((n, 3))]
        out.update(g_xy=g[0], g_conic=g[1], g_opacity=g[2], g_rgb=g[3])
    rc = lib.oracle_composite(n, _p(xy), _p(conic), _p(op), _p(rgb), _p(depth), _p(valid), m, _p(px), _p(py),
                              _p(bg), float(alpha_min), float(alpha_max), float(t_min), int(bool(reverse_t)),
                              _p(gc), _p(color), _p(tf), _p(last), _p(cnt), _p(margin), _p(order),
                              _p(g[0]), _p(g[1]), _p(g[2]), _p(g[3]), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_composite failed ({rc})")
    return out


def pixel_grid(width: int, height: int):
    """Centres of every pixel, row-major: (j + 0.5, i + 0.5)."""
    jj, ii = np.meshgrid(np.arange(width), np.arange(height))
    return (jj.ravel() + 0.5).astype(np.float64), (ii.ravel() + 0.5).astype(np.float64)


def composite_image(splats: dict, width: int, height: int, bg=(0.0, 0.0, 0.0), grad_image=None, **kw):
    """Whole image: returns image [3,H,W], t_final [H,W], last_id [H,W], n_contrib, margin [H,W] (+ grads)."""
    px, py = pixel_grid(width, height)
    gc = None
    if grad_image is not None:
        gc = np.asarray(grad_image, np.float64).reshape(3, height * width).T
    r = composite(splats, px, py, bg, gc, **kw)
    r["image"] = r["color"].T.reshape(3, height, width)
    for k in ("t_final", "last_id", "n_contrib", "margin", "order_margin"):
        r[k] = r[k].reshape(height, width)
    return r
