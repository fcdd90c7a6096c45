"""Thin ctypes binding of the C ABI in include/omnitrack.h.

Argument marshalling only: every step of the tracking path runs in the HIP
kernels of libomnitrack.so.  torch is used for device memory and streams.
There is no fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libomnitrack.so")

OT_MAX_LEVELS = 8
OT_MAX_WIN = 31
OT_DEFAULT_MIN_EIG = 6.5025
ERRORS = {0: "OT_OK", -1: "OT_E_INVAL", -2: "OT_E_SHAPE", -3: "OT_E_WORKSPACE",
          -4: "OT_E_LAUNCH", -5: "OT_E_UNSUPPORTED"}

# Every symbol the header declares.
EXPORTS = ["ot_pyramid_bytes", "ot_pyramid_layout", "ot_pyramid_build", "ot_lk_track",
           "ot_lk_track_ex", "ot_lk_track_fb", "ot_lk_order", "ot_box_update", "ot_fb_gate", "ot_box_update_scaled", "ot_box_scaled_bytes",
           "ot_box_update_scaled_noalloc",
           "ot_iou_matrix", "ot_assign", "ot_track_update", "ot_working_level",
           "ot_tvl1_default_params", "ot_tvl1_bytes", "ot_tvl1_flow", "ot_tvl1_flow_async",
           "ot_tvl1_texture_bytes", "ot_tvl1_texture", "ot_tvl1_flow_tex", "ot_box_mean_flow",
           "ot_batch_table_bytes", "ot_batch_pack", "ot_batch_run", "ot_batch_run_stages",
           "ot_strerror", "ot_version"]

# Points per box the scaled box update takes (OT_SCALE_MAX_POINTS).
SCALE_MAX_POINTS = 6144


class OtError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {ERRORS.get(code, code)} ({code})")
        self.code = code


OT_PYR_GRADS = 1


class OtPyr(C.Structure):
    _fields_ = [("level", C.c_void_p * OT_MAX_LEVELS), ("w", C.c_int32 * OT_MAX_LEVELS),
                ("h", C.c_int32 * OT_MAX_LEVELS), ("pitch", C.c_int32 * OT_MAX_LEVELS),
                ("levels", C.c_int32), ("flags", C.c_int32),
                ("grad", C.c_void_p * OT_MAX_LEVELS), ("gpitch", C.c_int32 * OT_MAX_LEVELS)]


class OtLkOpts(C.Structure):
    _fields_ = [("min_eig", C.c_float), ("iters_out", C.c_void_p), ("lam_out", C.c_void_p),
                ("margin", C.c_int32), ("base_level", C.c_int32), ("order", C.c_void_p)]


class OtTvl1Params(C.Structure):
    _fields_ = [("levels", C.c_int32), ("warps", C.c_int32), ("iters", C.c_int32),
                ("lam", C.c_float), ("theta", C.c_float), ("tau", C.c_float), ("eps", C.c_float),
                ("alpha", C.c_float), ("theta_s", C.c_float), ("tau_s", C.c_float),
                ("iters_s", C.c_int32)]


class OtJob(C.Structure):
    _fields_ = [("prev", OtPyr), ("next_frame", C.c_void_p), ("next_pitch", C.c_int32),
                ("next_ws", C.c_void_p), ("next_ws_bytes", C.c_size_t), ("levels", C.c_int32),
                ("pts", C.c_void_p), ("n", C.c_int32), ("next_pts", C.c_void_p),
                ("status", C.c_void_p), ("err", C.c_void_p), ("boxes", C.c_void_p),
                ("m", C.c_int32), ("box_id", C.c_void_p), ("out_boxes", C.c_void_p),
                ("out_count", C.c_void_p)]


class OtBatchCfg(C.Structure):
    _fields_ = [("win", C.c_int32), ("iters", C.c_int32), ("eps", C.c_float),
                ("min_eig", C.c_float), ("margin", C.c_int32), ("lk_waves", C.c_int32),
                ("chunk", C.c_int32), ("max_jobs", C.c_int32), ("max_points", C.c_int32),
                ("max_boxes", C.c_int32), ("max_tiles", C.c_int32), ("max_levels", C.c_int32),
                ("exact_grids", C.c_int32), ("lk_wpg", C.c_int32), ("lk_ppw", C.c_int32)]


_lib = None


def lib():
    """Load libomnitrack.so (built by paper_1910_06017_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1910_06017_amd/build.py "
                               "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        P, i32, sz, f32 = C.c_void_p, C.c_int32, C.c_size_t, C.c_float
        PP = C.POINTER(OtPyr)
        L.ot_pyramid_bytes.argtypes = [i32, i32, i32, i32]
        L.ot_pyramid_bytes.restype = sz
        L.ot_pyramid_layout.argtypes = [P, i32, i32, i32, i32, P, sz, i32, PP]
        L.ot_pyramid_layout.restype = i32
        L.ot_pyramid_build.argtypes = [P, i32, i32, i32, i32, P, sz, i32, PP, P]
        L.ot_pyramid_build.restype = i32
        L.ot_lk_track.argtypes = [PP, PP, P, i32, i32, i32, i32, f32, P, P, P, P]
        L.ot_lk_track.restype = i32
        L.ot_lk_track_ex.argtypes = [PP, PP, P, i32, i32, i32, i32, f32, P, P, P,
                                     C.POINTER(OtLkOpts), P]
        L.ot_lk_track_ex.restype = i32
        L.ot_lk_track_fb.argtypes = [PP, PP, P, i32, i32, i32, i32, f32, P, P, P, P, P,
                                     f32, P, P, C.POINTER(OtLkOpts), P]
        L.ot_lk_track_fb.restype = i32
        L.ot_lk_order.argtypes = [P, i32, i32, P, P]
        L.ot_lk_order.restype = i32
        L.ot_box_update.argtypes = [P, i32, P, P, P, P, i32, P, P, P]
        L.ot_box_update.restype = i32
        L.ot_fb_gate.argtypes = [P, P, P, P, i32, f32, P, P, P]
        L.ot_fb_gate.restype = i32
        L.ot_box_update_scaled.argtypes = [P, i32, P, P, P, P, i32, P, P, P, P, sz, P]
        L.ot_box_update_scaled.restype = i32
        L.ot_box_scaled_bytes.argtypes = [i32]
        L.ot_box_scaled_bytes.restype = sz
        L.ot_box_update_scaled_noalloc.argtypes = [P, i32, P, P, P, P, i32, P, P, P, P]
        L.ot_box_update_scaled_noalloc.restype = i32
        L.ot_tvl1_default_params.argtypes = [C.POINTER(OtTvl1Params)]
        L.ot_tvl1_default_params.restype = None
        L.ot_tvl1_bytes.argtypes = [i32, i32]
        L.ot_tvl1_bytes.restype = sz
        L.ot_tvl1_flow.argtypes = [PP, PP, C.POINTER(OtTvl1Params), P, sz, P, P]
        L.ot_tvl1_flow.restype = i32
        L.ot_tvl1_flow_async.argtypes = [PP, PP, C.POINTER(OtTvl1Params), P, sz, P, P, P]
        L.ot_tvl1_flow_async.restype = i32
        L.ot_tvl1_texture_bytes.argtypes = [i32, i32]
        L.ot_tvl1_texture_bytes.restype = sz
        L.ot_tvl1_texture.argtypes = [PP, C.POINTER(OtTvl1Params), P, sz, P]
        L.ot_tvl1_texture.restype = i32
        L.ot_tvl1_flow_tex.argtypes = [PP, PP, P, P, C.POINTER(OtTvl1Params), P, sz, P, P]
        L.ot_tvl1_flow_tex.restype = i32
        L.ot_box_mean_flow.argtypes = [P, i32, i32, P, i32, P, P, P]
        L.ot_box_mean_flow.restype = i32
        L.ot_working_level.argtypes = [i32, i32, i32]
        L.ot_working_level.restype = i32
        L.ot_iou_matrix.argtypes = [P, i32, P, i32, P, P, P]
        L.ot_iou_matrix.restype = i32
        L.ot_assign.argtypes = [P, i32, i32, f32, P, P, P]
        L.ot_assign.restype = i32
        L.ot_track_update.argtypes = [P, P, P, i32, i32, P, i32, P, P, P, P]
        L.ot_track_update.restype = i32
        L.ot_batch_table_bytes.argtypes = [C.POINTER(OtBatchCfg)]
        L.ot_batch_table_bytes.restype = sz
        L.ot_batch_pack.argtypes = [C.POINTER(OtJob), i32, C.POINTER(OtBatchCfg), P, sz, PP]
        L.ot_batch_pack.restype = i32
        L.ot_batch_run.argtypes = [P, P, sz, C.POINTER(OtBatchCfg), P]
        L.ot_batch_run.restype = i32
        L.ot_batch_run_stages.argtypes = [P, P, sz, C.POINTER(OtBatchCfg), i32, P]
        L.ot_batch_run_stages.restype = i32
        L.ot_strerror.argtypes = [i32]
        L.ot_strerror.restype = C.c_char_p
        L.ot_version.restype = i32
        _lib = L
    return _lib


def check(code: int, what: str) -> None:
    if code != 0:
        raise OtError(code, what)


# --------------------------------------------------------------------- torch side
def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _need(t, dtype, shape_last=None, what="tensor"):
    torch = _torch()
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous CUDA {dtype} tensor")
    if shape_last is not None and (t.dim() < 1 or t.shape[-1] != shape_last):
        raise ValueError(f"{what} must have last dimension {shape_last}")
    del torch


def pyramid_bytes(W: int, H: int, levels: int, flags: int = 0) -> int:
    return int(lib().ot_pyramid_bytes(W, H, levels, flags))


class Pyramid:
    """A device-resident pyramid: level 0 aliases `frame`, levels 1.. live in `ws`."""

    def __init__(self, frame, ws, desc: OtPyr):
        self.frame, self.ws, self.desc = frame, ws, desc

    @property
    def levels(self) -> int:
        return self.desc.levels

    def level(self, l: int):
        """Level l as an (h, w) uint8 tensor view (copies out of the pitched buffer)."""
        torch = _torch()
        if l == 0:
            return self.frame
        d = self.desc
        off = d.level[l] - self.ws.data_ptr()
        rows = self.ws[off:off + d.pitch[l] * d.h[l]].view(d.h[l], d.pitch[l])
        return rows[:, :d.w[l]]

    @property
    def has_grads(self) -> bool:
        return bool(self.desc.flags & OT_PYR_GRADS)

    def grads(self, l: int):
        """(sx, sy) int32 tensors of level l's materialized Scharr sums."""
        torch = _torch()
        d = self.desc
        if not self.has_grads:
            raise ValueError("pyramid was built without OT_PYR_GRADS")
        off = d.grad[l] - self.ws.data_ptr()
        words = self.ws[off:off + 4 * d.gpitch[l] * d.h[l]].view(torch.int32)
        v = words.view(d.h[l], d.gpitch[l])[:, :d.w[l]]
        sx = (v << 16) >> 16          # sign-extend the low half
        sy = v >> 16
        return sx, sy


def alloc_workspace(W: int, H: int, levels: int, device="cuda", grads: bool = False):
    torch = _torch()
    nb = pyramid_bytes(W, H, levels, OT_PYR_GRADS if grads else 0)
    # torch's caching allocator hands out 512-byte aligned blocks
    return torch.empty(max(nb, 256), dtype=torch.uint8, device=device)


def pyramid_build(frame, levels: int, ws=None, stream=None, grads: bool = False) -> Pyramid:
    """Build levels 1..levels-1 of `frame` ((H, W) uint8 CUDA tensor); with
    `grads` also the Scharr gradient planes of every level."""
    torch = _torch()
    _need(frame, torch.uint8, what="frame")
    H, W = frame.shape
    if ws is None:
        ws = alloc_workspace(W, H, levels, frame.device, grads=grads)
    desc = OtPyr()
    flags = OT_PYR_GRADS if grads else 0
    check(lib().ot_pyramid_build(_ptr(frame), W, H, frame.stride(0), levels, _ptr(ws), ws.numel(),
                                 flags, C.byref(desc), _stream_handle(stream)), "ot_pyramid_build")
    return Pyramid(frame, ws, desc)


def pyramid_layout(frame, levels: int, ws, grads: bool = False) -> Pyramid:
    H, W = frame.shape
    desc = OtPyr()
    check(lib().ot_pyramid_layout(_ptr(frame), W, H, frame.stride(0), levels, _ptr(ws),
                                  ws.numel(), OT_PYR_GRADS if grads else 0, C.byref(desc)),
          "ot_pyramid_layout")
    return Pyramid(frame, ws, desc)


def lk_track(prev: Pyramid, nxt: Pyramid, pts, win: int = 21, levels: int | None = None,
             iters: int = 30, eps: float = 0.01, min_eig: float = OT_DEFAULT_MIN_EIG,
             margin: int = 0, want_err: bool = True, want_diag: bool = False, out=None,
             stream=None, base_level: int = 0, order=None, iters_out=None):
    """Track (n, 2) float32 points.  Returns (next_pts, status, err[, iters, lam]).
    base_level > 0 tracks at that working level (levels base_level.. of both
    pyramids); points stay in level-0 pixels.  order: (n,) int32 processing
    order (see lk_order); iters_out: (n, levels) uint8 receiving the per-level
    iteration counts (without the other diagnostics)."""
    torch = _torch()
    _need(pts, torch.float32, 2, "pts")
    n = pts.shape[0]
    L = prev.levels - base_level if levels is None else levels
    dev = pts.device
    if out is None:
        next_pts = torch.empty((n, 2), dtype=torch.float32, device=dev)
        status = torch.empty(n, dtype=torch.uint8, device=dev)
        err = torch.empty(n, dtype=torch.float32, device=dev) if want_err else None
    else:
        next_pts, status, err = out
    opts = OtLkOpts(min_eig, None, None, margin, base_level, None)
    if order is not None:
        _need(order, torch.int32, None, "order")
        if order.numel() != n:
            raise ValueError("order must hold n entries")
        opts.order = _ptr(order)
    if iters_out is not None:
        _need(iters_out, torch.uint8, L, "iters_out")
        if iters_out.shape[0] != n:
            raise ValueError("iters_out must be (n, levels)")
        opts.iters_out = _ptr(iters_out)
    it = lam = None
    if want_diag:
        it = torch.zeros((n, L), dtype=torch.uint8, device=dev)
        lam = torch.zeros((n, L), dtype=torch.float32, device=dev)
        opts.iters_out, opts.lam_out = _ptr(it), _ptr(lam)
    check(lib().ot_lk_track_ex(C.byref(prev.desc), C.byref(nxt.desc), _ptr(pts), n, win, L,
                               iters, eps, _ptr(next_pts), _ptr(status), _ptr(err),
                               C.byref(opts), _stream_handle(stream)), "ot_lk_track")
    if want_diag:
        return next_pts, status, err, it, lam
    return next_pts, status, err


def lk_track_fb(prev: Pyramid, nxt: Pyramid, pts, win: int = 21, levels: int | None = None,
                iters: int = 30, eps: float = 0.01, min_eig: float = OT_DEFAULT_MIN_EIG,
                margin: int = 0, want_err: bool = True, out=None, stream=None,
                base_level: int = 0, fb_max: float | None = None, gate_out=None):
    """Track (n, 2) float32 points forward (prev -> nxt) and their forward
    results back (nxt -> prev) in one launch.  Returns (next_pts, status,
    err, back_pts, back_status), each as lk_track would give it; out, if
    given, is that 5-tuple of buffers (err may be None).  With fb_max the
    forward-backward gate follows in the same launch and (kept, fb_err), as
    fb_gate would give them, are appended (gate_out: that pair of buffers)."""
    torch = _torch()
    _need(pts, torch.float32, 2, "pts")
    n = pts.shape[0]
    L = prev.levels - base_level if levels is None else levels
    dev = pts.device
    if out is None:
        next_pts = torch.empty((n, 2), dtype=torch.float32, device=dev)
        status = torch.empty(n, dtype=torch.uint8, device=dev)
        err = torch.empty(n, dtype=torch.float32, device=dev) if want_err else None
        back_pts = torch.empty((n, 2), dtype=torch.float32, device=dev)
        back_status = torch.empty(n, dtype=torch.uint8, device=dev)
    else:
        next_pts, status, err, back_pts, back_status = out
    kept = fb_err = None
    if fb_max is not None:
        if gate_out is None:
            kept = torch.empty(n, dtype=torch.uint8, device=dev)
            fb_err = torch.empty(n, dtype=torch.float32, device=dev)
        else:
            kept, fb_err = gate_out
    opts = OtLkOpts(min_eig, None, None, margin, base_level, None)
    check(lib().ot_lk_track_fb(C.byref(prev.desc), C.byref(nxt.desc), _ptr(pts), n, win, L,
                               iters, eps, _ptr(next_pts), _ptr(status), _ptr(err),
                               _ptr(back_pts), _ptr(back_status),
                               0.0 if fb_max is None else fb_max, _ptr(fb_err), _ptr(kept),
                               C.byref(opts), _stream_handle(stream)), "ot_lk_track_fb")
    if fb_max is not None:
        return next_pts, status, err, back_pts, back_status, kept, fb_err
    return next_pts, status, err, back_pts, back_status


def lk_order(iters, out=None, stream=None):
    """Processing order of lk_track: the points of an (n, levels) uint8 table
    of iteration counts (an earlier pair of the same points) by descending
    total count; (n,) int32."""
    torch = _torch()
    _need(iters, torch.uint8, None, "iters")
    if iters.dim() != 2:
        raise ValueError("iters must be (n, levels)")
    n, L = iters.shape
    order = out if out is not None else torch.empty(n, dtype=torch.int32, device=iters.device)
    check(lib().ot_lk_order(_ptr(iters), n, L, _ptr(order), _stream_handle(stream)),
          "ot_lk_order")
    return order


def box_update(boxes, box_id, pts, next_pts, status, out=None, stream=None):
    """Per-box median displacement.  Returns (out_boxes (m,4), out_count (m,))."""
    torch = _torch()
    _need(boxes, torch.float32, 4, "boxes")
    m = boxes.shape[0]
    n = pts.shape[0]
    if out is None:
        ob = torch.empty((m, 4), dtype=torch.float32, device=boxes.device)
        oc = torch.empty(m, dtype=torch.int32, device=boxes.device)
    else:
        ob, oc = out
    check(lib().ot_box_update(_ptr(boxes), m, _ptr(box_id), _ptr(pts), _ptr(next_pts),
                              _ptr(status), n, _ptr(ob), _ptr(oc), _stream_handle(stream)),
          "ot_box_update")
    return ob, oc


def fb_gate(pts, back_pts, st_fwd, st_bwd, fb_max: float, want_err: bool = True,
            out=None, stream=None):
    """Forward-backward gate.  Returns (status (n,) uint8, fb_err (n,) float32
    or None): a point keeps status 1 when both tracks succeeded and
    |pts - back_pts| <= fb_max; fb_err is -1 where a track failed."""
    torch = _torch()
    _need(pts, torch.float32, 2, "pts")
    _need(back_pts, torch.float32, 2, "back_pts")
    _need(st_fwd, torch.uint8, None, "st_fwd")
    _need(st_bwd, torch.uint8, None, "st_bwd")
    n = pts.shape[0]
    if back_pts.shape[0] != n or st_fwd.numel() != n or st_bwd.numel() != n:
        raise ValueError("fb_gate: pts, back_pts, st_fwd and st_bwd must hold n points")
    if out is None:
        st = torch.empty(n, dtype=torch.uint8, device=pts.device)
        fe = torch.empty(n, dtype=torch.float32, device=pts.device) if want_err else None
    else:
        st, fe = out
    check(lib().ot_fb_gate(_ptr(pts), _ptr(back_pts), _ptr(st_fwd), _ptr(st_bwd), n,
                           float(fb_max), _ptr(fe) if fe is not None else None, _ptr(st),
                           _stream_handle(stream)), "ot_fb_gate")
    return st, fe


def box_scaled_workspace(m: int, device="cuda"):
    """Workspace for box_update_scaled on m boxes."""
    torch = _torch()
    return torch.empty(max(1, int(lib().ot_box_scaled_bytes(m))), dtype=torch.uint8, device=device)


def box_update_scaled(boxes, box_id, pts, next_pts, status, out=None, ws=None, stream=None):
    """Median-Flow box update: the centre moves by the median displacement
    and the half-extents scale by the median pairwise distance ratio.
    Returns (out_boxes (m,4), out_count (m,), out_scale (m,))."""
    torch = _torch()
    _need(boxes, torch.float32, 4, "boxes")
    _need(pts, torch.float32, 2, "pts")
    _need(next_pts, torch.float32, 2, "next_pts")
    _need(box_id, torch.int32, None, "box_id")
    _need(status, torch.uint8, None, "status")
    m = boxes.shape[0]
    n = pts.shape[0]
    if next_pts.shape[0] != n or box_id.numel() != n or status.numel() != n:
        raise ValueError("box_update_scaled: pts, next_pts, box_id and status must hold n points")
    if out is None:
        ob = torch.empty((m, 4), dtype=torch.float32, device=boxes.device)
        oc = torch.empty(m, dtype=torch.int32, device=boxes.device)
        os_ = torch.empty(m, dtype=torch.float32, device=boxes.device)
    else:
        ob, oc, os_ = out
    if ws is None:
        ws = box_scaled_workspace(m, boxes.device)
    check(lib().ot_box_update_scaled(_ptr(boxes), m, _ptr(box_id), _ptr(pts), _ptr(next_pts),
                                     _ptr(status), n, _ptr(ob), _ptr(oc), _ptr(os_), _ptr(ws),
                                     ws.numel() * ws.element_size(), _stream_handle(stream)),
          "ot_box_update_scaled")
    return ob, oc, os_


# Largest box count of the allocation-free scaled update.
SCALED_NOALLOC_MAX_BOXES = 64


def box_update_scaled_noalloc(boxes, box_id, pts, next_pts, status, out, stream=None):
    """box_update_scaled on the library's static device scratch: nothing is
    allocated, so the outputs (out_boxes m x 4, out_count m, out_scale m)
    must be given.  Calls on one GPU share the scratch: serialise them."""
    torch = _torch()
    _need(boxes, torch.float32, 4, "boxes")
    _need(pts, torch.float32, 2, "pts")
    _need(next_pts, torch.float32, 2, "next_pts")
    _need(box_id, torch.int32, None, "box_id")
    _need(status, torch.uint8, None, "status")
    m, n = boxes.shape[0], pts.shape[0]
    if next_pts.shape[0] != n or box_id.numel() != n or status.numel() != n:
        raise ValueError("box_update_scaled_noalloc: pts, next_pts, box_id and status must hold "
                         "n points")
    ob, oc, os_ = out
    check(lib().ot_box_update_scaled_noalloc(_ptr(boxes), m, _ptr(box_id), _ptr(pts),
                                             _ptr(next_pts), _ptr(status), n, _ptr(ob), _ptr(oc),
                                             _ptr(os_), _stream_handle(stream)),
          "ot_box_update_scaled_noalloc")
    return ob, oc, os_


def working_level(W: int, H: int, max_width: int = 1280) -> int:
    """The working level for a W x H frame (smallest level at most max_width wide)."""
    return int(lib().ot_working_level(W, H, max_width))


def tvl1_params(**kw) -> OtTvl1Params:
    """The library's TV-L1 defaults with the given fields replaced."""
    p = OtTvl1Params()
    lib().ot_tvl1_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise ValueError(f"unknown TV-L1 parameter {k}")
        setattr(p, k, v)
    return p


def tvl1_flow(prev: Pyramid, nxt: Pyramid, params: OtTvl1Params | None = None, ws=None,
              out=None, stream=None, aux_stream=None):
    """Dense TV-L1 flow at level 0: (H, W, 2) float32 (u_x, u_y) per pixel.
    With aux_stream, the structure-texture split runs there, ahead of the
    flow on `stream` (ot_tvl1_flow_async; the same result)."""
    torch = _torch()
    p = tvl1_params() if params is None else params
    W, H = prev.desc.w[0], prev.desc.h[0]
    need = int(lib().ot_tvl1_bytes(W, H))
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=prev.frame.device)
    flow = torch.empty((H, W, 2), dtype=torch.float32, device=prev.frame.device) if out is None else out
    args = (C.byref(prev.desc), C.byref(nxt.desc), C.byref(p), _ptr(ws),
            ws.numel() * ws.element_size(), _ptr(flow), _stream_handle(stream))
    if aux_stream is None:
        check(lib().ot_tvl1_flow(*args), "ot_tvl1_flow")
    else:
        check(lib().ot_tvl1_flow_async(*args, _stream_handle(aux_stream)), "ot_tvl1_flow_async")
    return flow


def tvl1_texture(pyr: Pyramid, params: OtTvl1Params | None = None, out=None, stream=None):
    """One frame's structure-texture buffer (opaque uint8 tensor) for
    tvl1_flow_tex: the texture and its gradient on every level."""
    torch = _torch()
    p = tvl1_params() if params is None else params
    W, H = pyr.desc.w[0], pyr.desc.h[0]
    need = int(lib().ot_tvl1_texture_bytes(W, H))
    tex = torch.empty(need, dtype=torch.uint8, device=pyr.frame.device) if out is None else out
    check(lib().ot_tvl1_texture(C.byref(pyr.desc), C.byref(p), _ptr(tex),
                                tex.numel() * tex.element_size(), _stream_handle(stream)),
          "ot_tvl1_texture")
    return tex


def tvl1_flow_tex(prev: Pyramid, nxt: Pyramid, prev_tex, next_tex,
                  params: OtTvl1Params | None = None, ws=None, out=None, stream=None):
    """tvl1_flow from two frames' texture buffers (tvl1_texture with the same
    parameters); the pyramids give the level sizes."""
    torch = _torch()
    p = tvl1_params() if params is None else params
    W, H = prev.desc.w[0], prev.desc.h[0]
    if ws is None:
        ws = torch.empty(int(lib().ot_tvl1_bytes(W, H)), dtype=torch.uint8, device=prev.frame.device)
    flow = torch.empty((H, W, 2), dtype=torch.float32, device=prev.frame.device) if out is None else out
    check(lib().ot_tvl1_flow_tex(C.byref(prev.desc), C.byref(nxt.desc), _ptr(prev_tex),
                                 _ptr(next_tex), C.byref(p), _ptr(ws),
                                 ws.numel() * ws.element_size(), _ptr(flow),
                                 _stream_handle(stream)), "ot_tvl1_flow_tex")
    return flow


def box_mean_flow(flow, boxes, out=None, stream=None):
    """Boxes moved by the mean dense flow inside them: (out_boxes, count)."""
    torch = _torch()
    _need(flow, torch.float32, 2, "flow")
    _need(boxes, torch.float32, 4, "boxes")
    H, W = flow.shape[0], flow.shape[1]
    m = boxes.shape[0]
    if out is None:
        ob = torch.empty((m, 4), dtype=torch.float32, device=boxes.device)
        oc = torch.empty(m, dtype=torch.int32, device=boxes.device)
    else:
        ob, oc = out
    check(lib().ot_box_mean_flow(_ptr(flow), W, H, _ptr(boxes), m, _ptr(ob), _ptr(oc),
                                 _stream_handle(stream)), "ot_box_mean_flow")
    return ob, oc


def iou_matrix(S, D, active=None, out=None, stream=None):
    """(m, k) float32 IoU of the scene boxes S (m, 4) against the
    detections D (k, 4), on the GPU; rows of objects with active == 0 are 0."""
    torch = _torch()
    _need(S, torch.float32, 4, "S")
    _need(D, torch.float32, 4, "D")
    if active is not None:
        _need(active, torch.uint8, None, "active")
        if active.numel() != S.shape[0]:
            raise ValueError("active must hold one flag per object")
    m, k = S.shape[0], D.shape[0]
    iou = torch.empty((m, k), dtype=torch.float32, device=S.device) if out is None else out
    check(lib().ot_iou_matrix(_ptr(S), m, _ptr(D), k, _ptr(active), _ptr(iou),
                              _stream_handle(stream)), "ot_iou_matrix")
    return iou


def _np(a, dtype, what):
    import numpy as np
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags.c_contiguous):
        raise ValueError(f"{what} must be a C-contiguous numpy {np.dtype(dtype).name} array")
    return a.ctypes.data if a.size else None


def assign(iou, iou_min: float = 0.3):
    """Optimal one-to-one matching on a host (m, k) float32 IoU matrix (the
    host part of the matching phase).  Returns (s2d (m,), d2s (k,), score)."""
    import numpy as np
    m, k = iou.shape
    s2d = np.empty(m, np.int32)
    d2s = np.empty(k, np.int32)
    score = C.c_double(0.0)
    check(lib().ot_assign(_np(iou, np.float32, "iou"), m, k, float(iou_min),
                          _np(s2d, np.int32, "s2d"), _np(d2s, np.int32, "d2s"),
                          C.byref(score)), "ot_assign")
    return s2d, d2s, score.value


def track_update(boxes, ids, lost, m: int, det, s2d, d2s, next_id: int):
    """Host update phase in place on capacity-sized arrays boxes (cap, 4)
    float32, ids (cap,) int32, lost (cap,) uint8 whose first m entries are
    the objects.  Returns (new object count, next id)."""
    import numpy as np
    cap = boxes.shape[0]
    if ids.shape[0] != cap or lost.shape[0] != cap or boxes.shape[1:] != (4,):
        raise ValueError("boxes, ids and lost must share one capacity")
    nid = C.c_int32(next_id)
    mo = C.c_int32(0)
    check(lib().ot_track_update(_np(boxes, np.float32, "boxes"), _np(ids, np.int32, "ids"),
                                _np(lost, np.uint8, "lost"), m, cap,
                                _np(det, np.float32, "det"), det.shape[0],
                                _np(s2d, np.int32, "s2d"), _np(d2s, np.int32, "d2s"),
                                C.byref(nid), C.byref(mo)), "ot_track_update")
    return mo.value, nid.value


def strerror(code: int) -> str:
    return lib().ot_strerror(code).decode()


def version() -> int:
    return int(lib().ot_version())
