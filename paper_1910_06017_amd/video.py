"""Tracking one video stream frame by frame, with the preprocessing of the
next frame prefetched (Sec. V-B).

Frames come from host memory (a decoder's output in pinned buffers).  Every
frame pair runs the three phases of the tracking stage (Sec. V-A): the
preprocessing (upload and Gaussian pyramid of the new frame), the feature
calculation (Lucas-Kanade at the resolution's working level) and the
prediction (per-box median); the caller receives each frame's boxes before
the next frame is tracked, as the matching and update phases need them.

With `prefetch`, frame t+1's upload and pyramid are enqueued on a second HIP
stream as soon as frame t's tracking has been, so they run while frame t is
tracked and its boxes come back; an event orders frame t+1's tracking after
its pyramid.  Without it, every step runs on one stream.  With `order`, the
points of a pair are tracked longest-first by their iteration counts in the
previous pair (a point keeps its index from frame to frame until the next
re-seed), which shortens the launch's tail.  The kernels and their inputs are
the same either way, so the results are identical.

Frame buffers and pyramid workspaces form a ring of three: frame t lives in
slot t % 3, which the pairs (t - 1, t) and (t, t + 1) read; frame t + 3
rewrites it only after the tracking of the pair (t, t + 1) has finished on
the device (an event wait on the preprocessing stream).

DenseVideoTracker is the same loop for the paper's dense engine (Sec. IV):
a frame's preprocessing is its upload, pyramid and structure-texture split,
computed once per frame, and a pair computes only the TV-L1 flow from the
two frames' textures and the mean flow inside every box.
"""
from __future__ import annotations

import numpy as np

from . import ops

__all__ = ["VideoTracker", "DenseVideoTracker"]


def _check_frames(frames, W: int, H: int) -> None:
    """Every frame must be a contiguous (H, W) uint8 host tensor: the upload
    copies H * W bytes from it into a device frame of that size."""
    import torch

    for t, f in enumerate(frames):
        if not isinstance(f, torch.Tensor) or f.dtype != torch.uint8 or f.device.type != "cpu":
            raise ValueError(f"frame {t}: expected a uint8 host tensor")
        if tuple(f.shape) != (H, W) or not f.is_contiguous():
            raise ValueError(f"frame {t}: expected a contiguous ({H}, {W}) tensor, "
                             f"got {tuple(f.shape)}")


def _check_boxes(bx: np.ndarray, t: int) -> None:
    if bx.ndim != 2 or bx.shape[1] != 4:
        raise ValueError(f"seeds[{t}]: boxes must be (m, 4)")


class VideoTracker:
    """Tracks the boxes of one stream through a sequence of frames.

    W, H: frame size; levels: tracking levels counted from the working
    level `base_level` (the pyramids hold base_level + levels levels);
    n_max / m_max: point and box capacities.  With `grads`, each frame's
    pyramid also gets its Scharr planes when it is built (on the
    preprocessing stream), and the pair that uses it as the first frame reads
    them instead of computing them (the same results, bit for bit)."""

    def __init__(self, W: int, H: int, levels: int, base_level: int = 0, n_max: int = 20000,
                 m_max: int = 64, win: int = 21, iters: int = 30, eps: float = 0.01,
                 prefetch: bool = True, order: bool = False, grads: bool = False,
                 device="cuda"):
        import torch

        from .serve import _copy  # noqa: F401  (host<->device copies without the dispatcher)

        self.torch = torch
        self.W, self.H, self.levels, self.base = W, H, levels, base_level
        self.win, self.iters, self.eps = win, iters, eps
        self.prefetch = prefetch
        self.dev = torch.device(device)
        PL = base_level + levels
        self.PL = PL
        self.frames = [torch.empty((H, W), dtype=torch.uint8, device=self.dev) for _ in range(3)]
        self.grads = grads
        self.ws = [ops.alloc_workspace(W, H, PL, self.dev, grads=grads) for _ in range(3)]
        self.pyr = [ops.pyramid_layout(self.frames[i], PL, self.ws[i], grads=grads)
                    for i in range(3)]
        n, m = max(1, n_max), max(1, m_max)
        self.n_max, self.m_max = n_max, m_max
        self.pts = [torch.zeros((n, 2), dtype=torch.float32, device=self.dev) for _ in range(2)]
        self.status = torch.zeros(n, dtype=torch.uint8, device=self.dev)
        self.err = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.box_id = torch.zeros(n, dtype=torch.int32, device=self.dev)
        self.boxes = [torch.zeros((m, 4), dtype=torch.float32, device=self.dev) for _ in range(2)]
        self.count = torch.zeros(m, dtype=torch.int32, device=self.dev)
        # per-point iteration counts of the last pair (two buffers) and the
        # processing order derived from them
        self.order = order
        self.iters_buf = [torch.zeros((n, levels), dtype=torch.uint8, device=self.dev)
                          for _ in range(2)]
        self.order_buf = torch.zeros(n, dtype=torch.int32, device=self.dev)
        self.host_boxes = torch.zeros((m, 4), dtype=torch.float32, pin_memory=True)
        self.host_count = torch.zeros(m, dtype=torch.int32, pin_memory=True)
        # both streams at the default priority
        self.s_pre = torch.cuda.Stream(self.dev)
        self.s_trk = torch.cuda.Stream(self.dev) if prefetch else self.s_pre
        torch.cuda.synchronize(self.dev)

    def _preprocess(self, frame, t: int, after_track):
        """Upload frame t into slot t % 3 and build its pyramid on the
        preprocessing stream, after `after_track` (the event of the last
        tracking that reads the slot), if any."""
        from .serve import _H2D, _copy

        i = t % 3
        sp = self.s_pre
        if after_track is not None:
            sp.wait_event(after_track)
        _copy(self.frames[i].data_ptr(), frame.data_ptr(), frame.numel(), _H2D,
              int(sp.cuda_stream))
        ops.pyramid_build(self.frames[i], self.PL, ws=self.ws[i], stream=sp, grads=self.grads)
        ev = self.torch.cuda.Event()
        ev.record(sp)
        return ev

    def track(self, frames: list, seeds: dict) -> list:
        """frames: (H, W) uint8 pinned host tensors.  seeds[t] = (pts (n, 2)
        float32, box_id (n,) int32, boxes (m, 4) float32): detections at frame
        t, which replace the points and boxes tracked from frame t (frame 0
        must have one).  Returns, for every t >= 1, (boxes (m, 4), counts (m,))
        predicted for frame t."""
        from .serve import _D2H, _H2D, _copy

        torch = self.torch
        if 0 not in seeds:
            raise ValueError("frame 0 needs detections")
        _check_frames(frames, self.W, self.H)
        T = len(frames)
        out = []
        pre_ev = [None] * T        # pyramid of frame t built
        trk_ev = [None] * T        # tracking of the pair (t-1, t) done
        pre_ev[0] = self._preprocess(frames[0], 0, None)
        if self.prefetch and T > 1:
            pre_ev[1] = self._preprocess(frames[1], 1, None)
        n = m = 0
        st = self.s_trk
        sh = int(st.cuda_stream)
        counts_valid = False   # iters_buf[cur] holds the last pair's counts of these points
        for t in range(1, T + 1):
            cur = (t - 1) & 1      # point / box buffers of frame t-1
            if t - 1 in seeds:
                counts_valid = False
                pts, bid, bx = (np.ascontiguousarray(a) for a in seeds[t - 1])
                n, m = len(pts), len(bx)
                if n > self.n_max or m > self.m_max:
                    raise ValueError("detections exceed the tracker's capacity")
                if pts.shape != (n, 2) or bid.shape != (n,):
                    raise ValueError(f"seeds[{t - 1}]: points must be (n, 2) with (n,) box ids")
                _check_boxes(bx, t - 1)
                pts = pts.astype(np.float32, copy=False)
                bid = bid.astype(np.int32, copy=False)
                bx = bx.astype(np.float32, copy=False)
                # pageable sources: staged by the runtime before the call returns
                _copy(self.pts[cur].data_ptr(), pts.ctypes.data, pts.nbytes, _H2D, sh)
                _copy(self.box_id.data_ptr(), bid.ctypes.data, bid.nbytes, _H2D, sh)
                _copy(self.boxes[cur].data_ptr(), bx.ctypes.data, bx.nbytes, _H2D, sh)
            if t == T:
                break
            if not self.prefetch:
                # one stream: the new frame's preprocessing runs now, in line
                pre_ev[t] = self._preprocess(frames[t], t, None)
            st.wait_event(pre_ev[t])
            P, Q = self.pyr[(t - 1) % 3], self.pyr[t % 3]
            nxt = 1 - cur
            order = None
            if self.order and counts_valid and n:
                # long tracks of the last pair first (the points keep their indices)
                order = ops.lk_order(self.iters_buf[cur][:n], out=self.order_buf[:n], stream=st)
            ops.lk_track(P, Q, self.pts[cur][:n], win=self.win, levels=self.levels,
                         iters=self.iters, eps=self.eps, stream=st, base_level=self.base,
                         out=(self.pts[nxt][:n], self.status[:n], self.err[:n]), order=order,
                         iters_out=self.iters_buf[nxt][:n] if self.order else None)
            counts_valid = True
            ops.box_update(self.boxes[cur][:m], self.box_id[:n], self.pts[cur][:n],
                           self.pts[nxt][:n], self.status[:n],
                           out=(self.boxes[nxt][:m], self.count[:m]), stream=st)
            _copy(self.host_boxes.data_ptr(), self.boxes[nxt].data_ptr(), m * 16, _D2H, sh)
            _copy(self.host_count.data_ptr(), self.count.data_ptr(), m * 4, _D2H, sh)
            ev = torch.cuda.Event()
            ev.record(st)
            trk_ev[t] = ev
            if self.prefetch and t + 1 < T:
                # frame t+1 goes to slot (t+1) % 3 = (t-2) % 3, last read by the
                # tracking of the pair (t-2, t-1)
                pre_ev[t + 1] = self._preprocess(frames[t + 1], t + 1,
                                                 trk_ev[t - 1] if t >= 2 else None)
            ev.synchronize()
            out.append((self.host_boxes[:m].numpy().copy(), self.host_count[:m].numpy().copy()))
        return out


class DenseVideoTracker:
    """Dense TV-L1 tracking of one video stream frame by frame (Sec. IV, V).

    Each frame's preprocessing (upload, pyramid, structure-texture split of
    every level) is computed once, when the frame arrives; the pair (t, t+1)
    then computes only the flow from frame t's and frame t+1's texture
    buffers, and every box moves by the mean flow inside it.  With `prefetch`,
    frame t+1's preprocessing runs on a second HIP stream while the pair
    (t-1, t) is tracked.  Frames, pyramids and texture buffers form a ring of
    three, ordered as in VideoTracker.  The flow is bit for bit the pairwise
    ot_tvl1_flow of the two frames."""

    def __init__(self, W: int, H: int, params=None, m_max: int = 64, prefetch: bool = True,
                 device="cuda"):
        import torch

        self.torch = torch
        self.W, self.H = W, H
        self.p = params if params is not None else ops.tvl1_params()
        self.prefetch = prefetch
        self.dev = torch.device(device)
        L = self.p.levels
        self.L = L
        self.frames = [torch.empty((H, W), dtype=torch.uint8, device=self.dev) for _ in range(3)]
        self.ws = [ops.alloc_workspace(W, H, L, self.dev) for _ in range(3)]
        self.pyr = [ops.pyramid_layout(self.frames[i], L, self.ws[i]) for i in range(3)]
        nt = int(ops.lib().ot_tvl1_texture_bytes(W, H))
        self.tex = [torch.empty(nt, dtype=torch.uint8, device=self.dev) for _ in range(3)]
        self.flow_ws = torch.empty(int(ops.lib().ot_tvl1_bytes(W, H)), dtype=torch.uint8,
                                   device=self.dev)
        self.flow = torch.empty((H, W, 2), dtype=torch.float32, device=self.dev)
        m = max(1, m_max)
        self.m_max = m_max
        self.boxes = [torch.zeros((m, 4), dtype=torch.float32, device=self.dev) for _ in range(2)]
        self.count = torch.zeros(m, dtype=torch.int32, device=self.dev)
        self.host_boxes = torch.zeros((m, 4), dtype=torch.float32, pin_memory=True)
        self.host_count = torch.zeros(m, dtype=torch.int32, pin_memory=True)
        # both streams at the default priority
        self.s_pre = torch.cuda.Stream(self.dev)
        self.s_trk = torch.cuda.Stream(self.dev) if prefetch else self.s_pre
        torch.cuda.synchronize(self.dev)

    def _preprocess(self, frame, t: int, after_track):
        from .serve import _H2D, _copy

        i = t % 3
        sp = self.s_pre
        if after_track is not None:
            sp.wait_event(after_track)
        _copy(self.frames[i].data_ptr(), frame.data_ptr(), frame.numel(), _H2D,
              int(sp.cuda_stream))
        ops.pyramid_build(self.frames[i], self.L, ws=self.ws[i], stream=sp)
        ops.tvl1_texture(self.pyr[i], self.p, out=self.tex[i], stream=sp)
        ev = self.torch.cuda.Event()
        ev.record(sp)
        return ev

    def track(self, frames: list, seeds: dict) -> list:
        """frames: (H, W) uint8 pinned host tensors.  seeds[t] = boxes (m, 4)
        float32 at frame t, which replace the boxes tracked to frame t (frame
        0 must have some).  Returns, for every t >= 1, (boxes (m, 4), counts
        (m,)) predicted for frame t."""
        from .serve import _D2H, _H2D, _copy

        torch = self.torch
        if 0 not in seeds:
            raise ValueError("frame 0 needs detections")
        _check_frames(frames, self.W, self.H)
        T = len(frames)
        out = []
        pre_ev = [None] * T
        trk_ev = [None] * T
        pre_ev[0] = self._preprocess(frames[0], 0, None)
        if self.prefetch and T > 1:
            pre_ev[1] = self._preprocess(frames[1], 1, None)
        m = 0
        st = self.s_trk
        sh = int(st.cuda_stream)
        for t in range(1, T + 1):
            cur = (t - 1) & 1
            if t - 1 in seeds:
                bx = np.ascontiguousarray(seeds[t - 1], dtype=np.float32)
                _check_boxes(bx, t - 1)
                m = len(bx)
                if m > self.m_max:
                    raise ValueError("detections exceed the tracker's capacity")
                _copy(self.boxes[cur].data_ptr(), bx.ctypes.data, bx.nbytes, _H2D, sh)
            if t == T:
                break
            if not self.prefetch:
                pre_ev[t] = self._preprocess(frames[t], t, None)
            st.wait_event(pre_ev[t])
            a, b = (t - 1) % 3, t % 3
            nxt = 1 - cur
            ops.tvl1_flow_tex(self.pyr[a], self.pyr[b], self.tex[a], self.tex[b], self.p,
                              ws=self.flow_ws, out=self.flow, stream=st)
            ops.box_mean_flow(self.flow, self.boxes[cur][:m],
                              out=(self.boxes[nxt][:m], self.count[:m]), stream=st)
            _copy(self.host_boxes.data_ptr(), self.boxes[nxt].data_ptr(), m * 16, _D2H, sh)
            _copy(self.host_count.data_ptr(), self.count.data_ptr(), m * 4, _D2H, sh)
            ev = torch.cuda.Event()
            ev.record(st)
            trk_ev[t] = ev
            if self.prefetch and t + 1 < T:
                # frame t+1 goes to slot (t+1) % 3, last read by the pair (t-2, t-1)
                pre_ev[t + 1] = self._preprocess(frames[t + 1], t + 1,
                                                 trk_ev[t - 1] if t >= 2 else None)
            ev.synchronize()
            out.append((self.host_boxes[:m].numpy().copy(), self.host_count[:m].numpy().copy()))
        return out
