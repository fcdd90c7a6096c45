"""CPU FP64 oracle of the pyramidal Lucas-Kanade box-tracking path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product path never imports it.  The C
library (`omnitrack_oracle.c`) shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "omnitrack_oracle.c")

from .matching import assign, iou, iou_matrix, track_update  # noqa: E402,F401
from .working import lk_track_working, working_level  # noqa: E402,F401
from . import tvl1  # noqa: E402,F401

GATE_MIN_EIG = 6.5025  # lambda_min / N threshold, (gray levels per pixel)^2 (= 1e-4 on [0,1])


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        compile_to(_SRC, LIB_PATH + ".tmp")
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None
_override = []


class use_library:
    """Context manager: route every wrapper call to another build of the
    oracle source (used by the tests that plant mistakes in a copy)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        _override.append(_load(self.path))
        return self

    def __exit__(self, *exc):
        _override.pop()
        return False


def compile_to(src: str, out: str) -> str:
    """Compile an oracle source file with the standard flags into `out`."""
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-I", _HERE, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def lib():
    global _lib
    if _override:
        return _override[-1]
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _load(LIB_PATH)
    return _lib


def _load(path: str):
    L = C.CDLL(path)
    P = C.c_void_p
    i32 = C.c_int32
    L.orc_level_dims.argtypes = [i32, i32, i32, P, P]
    L.orc_pyr_down.argtypes = [P, i32, i32, i32, P]
    L.orc_pyr_down_direct.argtypes = [P, i32, i32, i32, P]
    L.orc_pyramid.argtypes = [P, i32, i32, i32, i32, P]
    L.orc_scharr.argtypes = [P, i32, i32, P, P]
    L.orc_bilinear_u8.argtypes = [P, i32, i32, C.c_double, C.c_double]
    L.orc_bilinear_u8.restype = C.c_double
    L.orc_bilinear_i32.argtypes = [P, i32, i32, C.c_double, C.c_double]
    L.orc_bilinear_i32.restype = C.c_double
    L.orc_structure_tensor.argtypes = [P, i32, i32, C.c_double, C.c_double, i32, P]
    L.orc_structure_tensor.restype = C.c_double
    L.orc_min_eig.argtypes = [P]
    L.orc_min_eig.restype = C.c_double
    L.orc_lk_track.argtypes = [P, P, P, P, i32, P, i32, i32, i32, C.c_double, C.c_double,
                               P, P, P, P, P, P, i32]
    L.orc_lk_track.restype = i32
    L.orc_box_update.argtypes = [P, i32, P, P, P, P, i32, i32, P, P]
    L.orc_fb_gate.argtypes = [P, P, P, P, i32, C.c_double, P, P]
    L.orc_box_update_scaled.argtypes = [P, i32, P, P, P, P, i32, P, P, P]
    L.orc_max_threads.restype = i32
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def level_dims(W: int, H: int, levels: int):
    w = np.zeros(levels, np.int32)
    h = np.zeros(levels, np.int32)
    lib().orc_level_dims(W, H, levels, _p(w), _p(h))
    return [int(v) for v in w], [int(v) for v in h]


def pyr_down(img: np.ndarray, direct: bool = False) -> np.ndarray:
    img = np.ascontiguousarray(img, np.uint8)
    h, w = img.shape
    out = np.zeros(((h + 1) // 2, (w + 1) // 2), np.uint8)
    fn = lib().orc_pyr_down_direct if direct else lib().orc_pyr_down
    fn(_p(img), w, h, w, _p(out))
    return out


def pyramid(frame: np.ndarray, levels: int) -> list:
    """[level0, level1, ...] as separate tight uint8 arrays."""
    frame = np.ascontiguousarray(frame, np.uint8)
    H, W = frame.shape
    ws, hs = level_dims(W, H, levels)
    buf = np.zeros(sum(ws[l] * hs[l] for l in range(1, levels)) or 1, np.uint8)
    lib().orc_pyramid(_p(frame), W, H, W, levels, _p(buf))
    out, off = [frame], 0
    for l in range(1, levels):
        sz = ws[l] * hs[l]
        out.append(buf[off:off + sz].reshape(hs[l], ws[l]).copy())
        off += sz
    return out


def scharr(img: np.ndarray):
    """Integer Scharr responses (32 x gray levels per pixel): (sx, sy) int32."""
    img = np.ascontiguousarray(img, np.uint8)
    h, w = img.shape
    sx = np.zeros((h, w), np.int32)
    sy = np.zeros((h, w), np.int32)
    lib().orc_scharr(_p(img), w, h, _p(sx), _p(sy))
    return sx, sy


def bilinear(img: np.ndarray, x: float, y: float) -> float:
    h, w = img.shape
    if img.dtype == np.uint8:
        a = np.ascontiguousarray(img)
        return lib().orc_bilinear_u8(_p(a), w, h, float(x), float(y))
    a = np.ascontiguousarray(img, np.int32)
    return lib().orc_bilinear_i32(_p(a), w, h, float(x), float(y))


def structure_tensor(img: np.ndarray, cx: float, cy: float, win: int):
    """(G = [Gxx, Gxy, Gyy], lambda_min) for the window centred at (cx, cy)."""
    img = np.ascontiguousarray(img, np.uint8)
    h, w = img.shape
    G = np.zeros(3, np.float64)
    lam = lib().orc_structure_tensor(_p(img), w, h, float(cx), float(cy), int(win), _p(G))
    return G, lam


def min_eig(G) -> float:
    g = np.ascontiguousarray(G, np.float64)
    return lib().orc_min_eig(_p(g))


class LKResult:
    def __init__(self, next_pts, status, err, iters, lam, reason):
        self.next_pts, self.status, self.err = next_pts, status, err
        self.iters, self.lam, self.reason = iters, lam, reason


def lk_track_pyr(prev_pyr: list, next_pyr: list, pts: np.ndarray, win: int = 21,
                 levels: int | None = None, iters: int = 30, eps: float = 0.01,
                 min_eig: float = GATE_MIN_EIG, nthreads: int = 0) -> LKResult:
    """Track float32 points between two pyramids (lists of uint8 levels)."""
    if levels is None:
        levels = len(prev_pyr)
    prev = [np.ascontiguousarray(a, np.uint8) for a in prev_pyr[:levels]]
    nxt = [np.ascontiguousarray(a, np.uint8) for a in next_pyr[:levels]]
    for a, b in zip(prev, nxt):
        assert a.shape == b.shape
    w = np.array([a.shape[1] for a in prev], np.int32)
    h = np.array([a.shape[0] for a in prev], np.int32)
    pp = (C.c_void_p * levels)(*[a.ctypes.data for a in prev])
    pn = (C.c_void_p * levels)(*[a.ctypes.data for a in nxt])
    pts = np.ascontiguousarray(pts, np.float32).reshape(-1, 2)
    n = pts.shape[0]
    nxt_pts = np.zeros((n, 2), np.float64)
    status = np.zeros(n, np.uint8)
    err = np.zeros(n, np.float64)
    it = np.zeros((n, levels), np.int32)
    lam = np.zeros((n, levels), np.float64)
    reason = np.zeros(n, np.int32)
    rc = lib().orc_lk_track(C.cast(pp, C.c_void_p), C.cast(pn, C.c_void_p), _p(w), _p(h),
                            levels, _p(pts), n, win, iters, eps, min_eig, _p(nxt_pts),
                            _p(status), _p(err), _p(it), _p(lam), _p(reason), nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return LKResult(nxt_pts, status, err, it, lam, reason)


def lk_track(frame0: np.ndarray, frame1: np.ndarray, pts: np.ndarray, win: int = 21,
             levels: int = 4, iters: int = 30, eps: float = 0.01,
             min_eig: float = GATE_MIN_EIG, nthreads: int = 0) -> LKResult:
    """Build both pyramids and track (the whole per-frame-pair path on the CPU)."""
    return lk_track_pyr(pyramid(frame0, levels), pyramid(frame1, levels), pts, win, levels,
                        iters, eps, min_eig, nthreads)


def box_update(boxes, box_id, pts, next_pts, status, use_mean: bool = False):
    """(out_boxes float64 (m,4), out_count int32 (m,))."""
    boxes = np.ascontiguousarray(boxes, np.float64).reshape(-1, 4)
    m = boxes.shape[0]
    box_id = np.ascontiguousarray(box_id, np.int32)
    pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 2)
    next_pts = np.ascontiguousarray(next_pts, np.float64).reshape(-1, 2)
    status = np.ascontiguousarray(status, np.uint8)
    n = pts.shape[0]
    out = np.zeros((m, 4), np.float64)
    cnt = np.zeros(m, np.int32)
    lib().orc_box_update(_p(boxes), m, _p(box_id), _p(pts), _p(next_pts), _p(status), n,
                         int(use_mean), _p(out), _p(cnt))
    return out, cnt


def fb_gate(pts, back_pts, st_fwd, st_bwd, fb_max: float):
    """Forward-backward check: (fb_err float64 (n,), status uint8 (n,))."""
    pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 2)
    back = np.ascontiguousarray(back_pts, np.float64).reshape(-1, 2)
    sf = np.ascontiguousarray(st_fwd, np.uint8)
    sb = np.ascontiguousarray(st_bwd, np.uint8)
    n = pts.shape[0]
    err = np.zeros(n, np.float64)
    st = np.zeros(n, np.uint8)
    lib().orc_fb_gate(_p(pts), _p(back), _p(sf), _p(sb), n, float(fb_max), _p(err), _p(st))
    return err, st


def box_update_scaled(boxes, box_id, pts, next_pts, status):
    """Median-Flow box update: (out_boxes (m,4), out_count (m,), scale (m,))."""
    boxes = np.ascontiguousarray(boxes, np.float64).reshape(-1, 4)
    m = boxes.shape[0]
    box_id = np.ascontiguousarray(box_id, np.int32)
    pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 2)
    next_pts = np.ascontiguousarray(next_pts, np.float64).reshape(-1, 2)
    status = np.ascontiguousarray(status, np.uint8)
    n = pts.shape[0]
    out = np.zeros((m, 4), np.float64)
    cnt = np.zeros(m, np.int32)
    scale = np.zeros(m, np.float64)
    lib().orc_box_update_scaled(_p(boxes), m, _p(box_id), _p(pts), _p(next_pts), _p(status), n,
                                _p(out), _p(cnt), _p(scale))
    return out, cnt, scale


def max_threads() -> int:
    return int(lib().orc_max_threads())
