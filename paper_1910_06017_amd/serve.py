"""Continuous-batching serving loop for many video streams on one GPU.

Frames arrive per stream at their own times.  The scheduler admits a stream
when its resident state fits the HBM budget (otherwise it waits in FIFO
order), and every tick batches the oldest waiting frame of every admitted
stream into one batched launch (new pyramid, tracking, box update; see
`batch.py`).  Frames that arrive while a tick runs join the next tick.  A
stream's previous pyramid, points and boxes stay resident between frames:
each frame builds one pyramid and the two pyramid workspaces swap roles.
A frame may carry synthetic "detections" (the benchmark attaches them to
every 10th frame of a stream) that replace the stream's boxes and points.  Streams silent for `evict_after` seconds are evicted
and their memory returned to the budget.

`Scheduler` is pure Python (no GPU) so admission, batching order and
eviction are testable with a fake clock and a fake executor; `GpuExecutor`
runs ticks on the device through the C ABI, and `PlainExecutor` processes
the same frames one at a time with the per-stream calls for comparison.
"""
from __future__ import annotations

import gc
import math
import time
from collections import deque
from dataclasses import dataclass

import numpy as np

__all__ = ["StreamSpec", "Frame", "Result", "Scheduler", "GpuExecutor", "PlainExecutor",
           "make_trace", "run_trace", "stream_footprint", "latency_stats"]


@dataclass
class StreamSpec:
    sid: int
    W: int
    H: int
    levels: int
    n_max: int          # points capacity
    m_max: int          # boxes capacity


@dataclass
class Frame:
    sid: int
    k: int               # frame index within the stream
    t_arrival: float
    pixels: object       # (H, W) uint8 host array (pinned torch tensor or numpy)
    reseed: object = None  # (pts float32 n x 2, box_id int32 n, boxes float32 m x 4) or None


def check_frame(fr: Frame, spec: StreamSpec) -> None:
    """A frame must carry H * W uint8 pixels in one contiguous (H, W) host
    array, and detections of the documented shapes within the stream's
    capacities: the uploads copy that many bytes into device buffers sized
    by the spec.  Raises ValueError."""
    px = fr.pixels
    if hasattr(px, "data_ptr"):
        import torch

        ok = (px.dtype == torch.uint8 and px.device.type == "cpu" and px.is_contiguous()
              and tuple(px.shape) == (spec.H, spec.W))
    else:
        ok = (isinstance(px, np.ndarray) and px.dtype == np.uint8
              and px.shape == (spec.H, spec.W))
    if not ok:
        raise ValueError(f"stream {fr.sid} frame {fr.k}: pixels must be a contiguous "
                         f"({spec.H}, {spec.W}) uint8 host array")
    if fr.reseed is not None:
        pts, bid, bx = (np.asarray(a) for a in fr.reseed)
        n, m = len(pts), len(bx)
        if pts.shape != (n, 2) or bid.shape != (n,) or bx.shape != (m, 4):
            raise ValueError(f"stream {fr.sid} frame {fr.k}: detections must be points (n, 2), "
                             "box ids (n,) and boxes (m, 4)")
        if n > spec.n_max or m > spec.m_max:
            raise ValueError(f"stream {fr.sid} frame {fr.k}: detections exceed the stream's capacity")


@dataclass
class Result:
    sid: int
    k: int
    t_arrival: float
    t_done: float
    boxes: np.ndarray    # (m, 4) float32 predicted boxes (empty for a stream's first frame)
    counts: np.ndarray   # (m,) int32 tracked points per box
    tick: int = -1

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def stream_footprint(spec: StreamSpec) -> int:
    """Resident device bytes of one stream: two frames, two pyramid
    workspaces, points and outputs (~25 B per point), boxes."""
    from . import ops

    frames = 2 * spec.W * spec.H
    pyr = 2 * max(256, ops.pyramid_bytes(spec.W, spec.H, spec.levels))
    pts = spec.n_max * (8 + 8 + 1 + 4 + 4)
    boxes = spec.m_max * (16 + 16 + 4)
    return frames + pyr + pts + boxes


class Scheduler:
    """Admission by HBM budget, continuous batching, eviction (no GPU)."""

    # silence is checked at most this often (eviction waits `evict_after`, seconds)
    EVICT_CHECK_S = 0.005

    def __init__(self, budget: int, max_jobs: int, max_points: int, evict_after: float = 2.0,
                 footprint=stream_footprint):
        self.budget, self.max_jobs, self.max_points = budget, max_jobs, max_points
        self.evict_after = evict_after
        self.footprint = footprint
        self.specs: dict = {}
        self.admitted: dict = {}     # sid -> bytes
        self.waiting: deque = deque()  # sids waiting for admission, FIFO
        self.queues: dict = {}       # sid -> deque of frames
        self.nonempty: set = set()   # sids with queued frames
        self.npending = 0
        self.last_seen: dict = {}
        self.used = 0
        self.evicted: list = []
        self.rejected: list = []
        self._next_evict_check = -math.inf

    def register(self, spec: StreamSpec):
        self.specs[spec.sid] = spec
        self.queues.setdefault(spec.sid, deque())

    def arrive(self, fr: Frame):
        q = self.queues[fr.sid]
        q.append(fr)
        self.npending += 1
        self.nonempty.add(fr.sid)
        self.last_seen[fr.sid] = fr.t_arrival
        if fr.sid not in self.admitted and fr.sid not in self.waiting:
            fp = self.footprint(self.specs[fr.sid])
            if fp > self.budget:
                self.rejected.append(fr.sid)   # can never fit
                self.npending -= len(q)
                q.clear()
                self.nonempty.discard(fr.sid)
                return
            self.waiting.append(fr.sid)

    def admit(self) -> list:
        """Admit waiting streams in FIFO order while they fit; returns newly admitted sids."""
        new = []
        while self.waiting:
            sid = self.waiting[0]
            fp = self.footprint(self.specs[sid])
            if self.used + fp > self.budget:
                break
            self.waiting.popleft()
            self.admitted[sid] = fp
            self.used += fp
            new.append(sid)
        return new

    def evict_idle(self, now: float) -> list:
        if now < self._next_evict_check:
            return []
        self._next_evict_check = now + self.EVICT_CHECK_S
        gone = []
        for sid in list(self.admitted):
            if not self.queues[sid] and now - self.last_seen.get(sid, now) > self.evict_after:
                self.used -= self.admitted.pop(sid)
                gone.append(sid)
        self.evicted += gone
        return gone

    def eviction_times(self, now: float) -> list:
        """When each idle admitted stream becomes evictable (no earlier than
        the next silence check)."""
        return [max(self.last_seen.get(sid, now) + self.evict_after, self._next_evict_check)
                for sid in self.admitted if not self.queues[sid]]

    def next_batch(self) -> list:
        """Oldest waiting frame of each admitted stream (oldest first), within
        the per-tick job and point capacities."""
        cands = [(self.queues[sid][0].t_arrival, sid) for sid in self.nonempty
                 if sid in self.admitted]
        cands.sort()
        batch, pts = [], 0
        for _, sid in cands:
            n = self.specs[sid].n_max
            if len(batch) >= self.max_jobs or pts + n > self.max_points:
                break
            q = self.queues[sid]
            batch.append(q.popleft())
            if not q:
                self.nonempty.discard(sid)
            pts += n
        self.npending -= len(batch)
        return batch

    def requeue(self, frames: list):
        """Put frames taken by next_batch back at the head of their queues."""
        for fr in reversed(frames):
            self.queues[fr.sid].appendleft(fr)
            self.nonempty.add(fr.sid)
            self.npending += 1

    def pending(self) -> int:
        return self.npending


# ----------------------------------------------------------------------------- GPU side
_HIP = None


def _hip():
    """hipMemcpyAsync from the HIP runtime (host<->device copies without the
    torch dispatcher on the per-frame path)."""
    global _HIP
    if _HIP is None:
        import ctypes as C

        h = C.CDLL("libamdhip64.so")
        h.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        h.hipMemcpyAsync.restype = C.c_int
        _HIP = h
    return _HIP


_H2D, _D2H = 1, 2
# stages of ot_batch_run_stages
OT_STAGE_PYRAMID, OT_STAGE_TRACK = 1, 2


def _copy(dst: int, src: int, nbytes: int, kind: int, stream: int):
    if nbytes:
        rc = _hip().hipMemcpyAsync(dst, src, nbytes, kind, stream)
        if rc != 0:
            raise RuntimeError(f"hipMemcpyAsync failed ({rc})")


class _Arena:
    """Per-executor result arenas: boxes (two parities) and counts per slot,
    device and pinned host, so one copy brings back every stream's result."""

    def __init__(self, torch, device, slots: int, m_chunk: int):
        self.m_chunk = m_chunk
        self.dev_boxes = [torch.zeros((slots * m_chunk, 4), dtype=torch.float32, device=device)
                          for _ in range(2)]
        self.dev_count = torch.zeros(slots * m_chunk, dtype=torch.int32, device=device)
        self.host_boxes = [torch.zeros((slots * m_chunk, 4), dtype=torch.float32, pin_memory=True)
                           for _ in range(2)]
        self.host_count = torch.zeros(slots * m_chunk, dtype=torch.int32, pin_memory=True)
        self.free = list(range(slots - 1, -1, -1))

    def take(self) -> int:
        if not self.free:
            raise RuntimeError("no result slot left (raise max_slots)")
        return self.free.pop()

    def give(self, k: int):
        self.free.append(k)


class _Slot:
    """Resident device state of one stream: three frames and pyramid
    workspaces (frame f in buffer f % 3, so the next frame's upload and
    pyramid can run while the current pair is tracked), two point buffers and
    two box chunks (frame f in f % 2), and the C job descriptors of every
    frame index mod 6, built once."""

    NF = 3   # frame / pyramid buffers
    NP = 2   # point / box buffers

    def __init__(self, spec: StreamSpec, device, arena: _Arena, stream=None):
        import ctypes as C

        import torch

        from . import ops

        if spec.m_max > arena.m_chunk:
            raise ValueError(f"stream {spec.sid}: {spec.m_max} boxes > {arena.m_chunk} per stream")
        self.spec = spec
        H, W, L = spec.H, spec.W, spec.levels
        n = max(1, spec.n_max)
        # allocated and initialised on the stream that will use them, so the
        # fills are ordered before the first upload or re-seed
        with torch.cuda.stream(stream) if stream is not None else _nullctx():
            self.frames = [torch.empty((H, W), dtype=torch.uint8, device=device)
                           for _ in range(self.NF)]
            self.ws = [ops.alloc_workspace(W, H, L, device) for _ in range(self.NF)]
            self.pts = [torch.zeros((n, 2), dtype=torch.float32, device=device)
                        for _ in range(self.NP)]
            self.status = torch.zeros(n, dtype=torch.uint8, device=device)
            self.err = torch.zeros(n, dtype=torch.float32, device=device)
            self.box_id = torch.full((n,), -1, dtype=torch.int32, device=device)
        self.arena = arena
        self.chunk = arena.take()
        c0 = self.chunk * arena.m_chunk
        self.c0 = c0
        self.boxes = [arena.dev_boxes[p][c0:c0 + arena.m_chunk] for p in range(self.NP)]
        self.count = arena.dev_count[c0:c0 + arena.m_chunk]
        self.pyr = [ops.pyramid_layout(self.frames[i], L, self.ws[i]) for i in range(self.NF)]
        # job[f % 6]: frame f uploaded into buffer f % 3 (previous: (f-1) % 3),
        # points and boxes from buffer (f-1) % 2 into f % 2
        self.job = []
        for f in range(self.NF * self.NP):
            j = ops.OtJob()
            fi, fq = f % self.NF, (f - 1) % self.NF
            p, q = f % self.NP, (f - 1) % self.NP
            j.prev = self.pyr[fq].desc
            j.next_frame = self.frames[fi].data_ptr()
            j.next_pitch = W
            j.next_ws = self.ws[fi].data_ptr()
            j.next_ws_bytes = self.ws[fi].numel()
            j.levels = L
            j.pts, j.next_pts = self.pts[q].data_ptr(), self.pts[p].data_ptr()
            j.status, j.err = self.status.data_ptr(), self.err.data_ptr()
            j.boxes, j.out_boxes = self.boxes[q].data_ptr(), self.boxes[p].data_ptr()
            j.box_id, j.out_count = self.box_id.data_ptr(), self.count.data_ptr()
            self.job.append(j)
        self.f = -1         # index of the last frame submitted
        self.n = 0
        self.m = 0
        self.frames_done = 0
        self._c = C

    @property
    def started(self) -> bool:
        return self.f >= 0

    def release(self):
        self.arena.give(self.chunk)

    def upload(self, fr: Frame, f: int, stream: int):
        check_frame(fr, self.spec)
        px = fr.pixels
        dst = self.frames[f % self.NF].data_ptr()
        if hasattr(px, "data_ptr"):
            _copy(dst, px.data_ptr(), px.numel(), _H2D, stream)
        else:
            a = np.ascontiguousarray(px, np.uint8)
            _copy(dst, a.ctypes.data, a.nbytes, _H2D, stream)

    def reseed(self, fr: Frame, f: int, stream: int):
        """Detections at frame f replace the points and boxes tracked from it,
        after the frame's own pair has been processed."""
        if fr.reseed is None:
            return
        pts, bid, bx = (np.ascontiguousarray(a) for a in fr.reseed)
        n, m = len(pts), len(bx)
        if n > self.spec.n_max or m > self.spec.m_max:
            raise ValueError("detections exceed the stream's capacity")
        pts = pts.astype(np.float32, copy=False)
        bid = bid.astype(np.int32, copy=False)
        bx = bx.astype(np.float32, copy=False)
        p = f % self.NP
        # pageable sources: the runtime stages them before the call returns
        _copy(self.pts[p].data_ptr(), pts.ctypes.data, pts.nbytes, _H2D, stream)
        _copy(self.box_id.data_ptr(), bid.ctypes.data, bid.nbytes, _H2D, stream)
        _copy(self.boxes[p].data_ptr(), bx.ctypes.data, bx.nbytes, _H2D, stream)
        self.n, self.m = n, m

    def job_for(self, f: int):
        """C job for frame f (no points or boxes on the stream's first frame)."""
        j = self.job[f % (self.NF * self.NP)]
        if f == 0 or not self.started:
            j.n = j.m = 0
        else:
            j.n, j.m = self.n, self.m
        return j


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False


class _Tick:
    __slots__ = ("idx", "metas", "ev_pre", "ev_trk", "ring", "spans", "t_done")

    def __init__(self, idx, metas, ev_pre, ev_trk, ring, spans):
        self.idx, self.metas, self.ev_pre, self.ev_trk = idx, metas, ev_pre, ev_trk
        self.ring, self.spans = ring, spans
        self.t_done = None   # when the host saw the tick complete


class GpuExecutor:
    """Runs ticks of frames (at most one per stream each) as batched launches,
    with up to `depth` ticks in flight on the device.

    A tick's preprocessing stage (frame uploads, the table copy, the pyramid
    launches) runs on one HIP stream and its tracking stage (tracking, box
    update, the copy back of the results, re-seeds) on a second one, after an
    event of the first: tick k+1's uploads and pyramids overlap tick k's
    tracking, and different streams' ticks overlap on the device.  Results
    are collected by event queries (`poll`), not by blocking each tick.

    Buffer reuse is ordered by events: tick k's preprocessing waits for the
    tracking stage of tick k - depth (its device table and the frame buffers
    it rewrites were last read there), and a stream's frame f reuses the frame
    buffer of frame f - 3, whose last reader (the pair f-2, f-1) lies in an
    earlier tick.  `depth=1` is the blocking loop: one tick at a time.

    A tick of a single frame (most ticks at light load) goes through the
    per-stream calls instead (`solo`): the same arithmetic without a table
    to pack and copy, and, when nothing else is in flight, on one stream."""

    def __init__(self, win=21, iters=30, eps=0.01, max_jobs=64, max_points=1 << 21,
                 max_boxes=4096, max_levels=5, schedule=None, device="cuda", max_slots=128,
                 m_chunk=64, depth=2, solo=True, solo_overlap=True):
        import torch

        from . import batch, ops

        if depth < 1 or depth > 2:
            raise ValueError("depth must be 1 or 2")
        self.torch = torch
        self.device = torch.device(device)
        sched = schedule or {}
        self.cfg = batch.BatchConfig(win=win, iters=iters, eps=eps, max_jobs=max_jobs,
                                     max_points=max_points, max_boxes=max_boxes,
                                     max_tiles=1 << 15, max_levels=max_levels, exact_grids=True,
                                     **sched)
        self.ccfg = self.cfg.to_c()
        import ctypes as C
        nb = int(ops.lib().ot_batch_table_bytes(C.byref(self.ccfg)))
        if nb == 0:
            raise ValueError("invalid batch configuration")
        self.table_bytes = nb
        self.depth = depth
        self.solo = solo     # one-frame ticks through the per-stream calls
        # a one-frame tick submitted while another runs: preprocessing on the
        # other stream (True) or everything behind it on the tracking stream
        self.solo_overlap = solo_overlap
        self.opts = ops.OtLkOpts(float(self.cfg.min_eig), None, None, self.cfg.margin, 0, None)
        self.host_tab = [torch.empty(nb, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
        self.dev_tab = [torch.empty(nb, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self.arena = _Arena(torch, self.device, max_slots, m_chunk)
        # host copies of the results of the ticks in flight (depth + 1 ring)
        self.ring_boxes = [[torch.zeros((max_slots * m_chunk, 4), dtype=torch.float32,
                                        pin_memory=True) for _ in range(2)]
                           for _ in range(depth + 1)]
        self.ring_count = [torch.zeros(max_slots * m_chunk, dtype=torch.int32, pin_memory=True)
                           for _ in range(depth + 1)]
        self.slots: dict = {}
        # both streams at the default priority
        self.s_pre = torch.cuda.Stream(self.device)
        self.s_trk = torch.cuda.Stream(self.device)
        self.h_pre = int(self.s_pre.cuda_stream)
        self.h_trk = int(self.s_trk.cuda_stream)
        self.inflight: deque = deque()
        self.trk_events: dict = {}   # tick index -> tracking-stage event
        self.ready: list = []        # results collected outside poll
        self.ticks = 0
        self._now = time.perf_counter
        torch.cuda.synchronize(self.device)  # the arena's fills precede both streams' work

    # -------------------------------------------------------------- slots
    def admit(self, spec: StreamSpec):
        self.slots[spec.sid] = _Slot(spec, self.device, self.arena, self.s_pre)
        # the slot's fills (on the preprocessing stream) precede any tracking
        self.s_trk.wait_stream(self.s_pre)

    def evict(self, sid: int):
        s = self.slots.pop(sid, None)
        if s is not None:
            # results of the ticks drained here are handed out by the next poll
            self.ready += self.drain()
            self.torch.cuda.synchronize(self.device)
            s.release()

    # -------------------------------------------------------------- pipeline
    def busy(self) -> bool:
        return bool(self.inflight)

    def can_submit(self) -> bool:
        return len(self.inflight) < self.depth

    def _observe(self):
        """Stamp the completion of the ticks in flight that have completed
        (tracking stages complete in submission order).  Called between the
        enqueue steps of a submit, so that a tick that completes while the
        host enqueues the next one is seen then, not when the submit returns."""
        for tk in self.inflight:
            if tk.t_done is not None:
                continue
            if not tk.ev_trk.query():
                return
            tk.t_done = self._now()

    def submit(self, frames: list, now=time.perf_counter):
        """Enqueue one tick of frames (at most one per stream).  `now` is the
        clock the completion times of the ticks in flight are read from."""
        import ctypes as C

        from . import ops

        torch = self.torch
        if not self.can_submit():
            raise RuntimeError("too many ticks in flight")
        for fr in frames:
            check_frame(fr, self.slots[fr.sid].spec)
        self._now = now
        if len(frames) == 1 and self.solo:
            self._submit_one(frames[0])
            return
        k = self.ticks
        t = k % 2
        L = ops.lib()
        metas, jobs = [], []
        for fr in frames:
            slot = self.slots[fr.sid]
            f = slot.f + 1
            jobs.append(slot.job_for(f))
            metas.append((fr, slot, f, slot.m if slot.started else 0))
        arr = (ops.OtJob * max(1, len(jobs)))()
        for i, j in enumerate(jobs):
            C.memmove(C.byref(arr, i * C.sizeof(ops.OtJob)), C.byref(j), C.sizeof(ops.OtJob))
        # host table t was last copied by tick k-2, which has completed (depth <= 2)
        ops.check(L.ot_batch_pack(arr, len(jobs), C.byref(self.ccfg),
                                  int(self.host_tab[t].data_ptr()), self.table_bytes, None),
                  "ot_batch_pack")
        # ---- preprocessing stage
        prior = self.trk_events.pop(k - self.depth, None)
        if prior is not None:
            self.s_pre.wait_event(prior)
        for fr, slot, f, _ in metas:
            slot.upload(fr, f, self.h_pre)
        self._observe()
        ops.check(L.ot_batch_run_stages(int(self.host_tab[t].data_ptr()),
                                        int(self.dev_tab[t].data_ptr()), self.table_bytes,
                                        C.byref(self.ccfg), OT_STAGE_PYRAMID, self.h_pre),
                  "ot_batch_run_stages(pyramid)")
        self._observe()
        ev_pre = torch.cuda.Event()
        ev_pre.record(self.s_pre)
        # ---- tracking stage
        self.s_trk.wait_event(ev_pre)
        ops.check(L.ot_batch_run_stages(int(self.host_tab[t].data_ptr()),
                                        int(self.dev_tab[t].data_ptr()), self.table_bytes,
                                        C.byref(self.ccfg), OT_STAGE_TRACK, self.h_trk),
                  "ot_batch_run_stages(track)")
        self._observe()
        r = k % (self.depth + 1)
        a = self.arena
        mc = a.m_chunk
        spans = {}
        for fr, slot, f, m in metas:
            if m:
                par = f % _Slot.NP
                lo, hi = spans.get(par, (slot.c0, slot.c0 + mc))
                spans[par] = (min(lo, slot.c0), max(hi, slot.c0 + mc))
        clo = min((lo for lo, _ in spans.values()), default=0)
        chi = max((hi for _, hi in spans.values()), default=0)
        for par, (lo, hi) in spans.items():
            _copy(self.ring_boxes[r][par][lo:].data_ptr(), a.dev_boxes[par][lo:].data_ptr(),
                  (hi - lo) * 16, _D2H, self.h_trk)
        if chi > clo:
            _copy(self.ring_count[r][clo:].data_ptr(), a.dev_count[clo:].data_ptr(),
                  (chi - clo) * 4, _D2H, self.h_trk)
        self._observe()
        for fr, slot, f, _ in metas:
            slot.reseed(fr, f, self.h_trk)
            slot.f = f
        ev_trk = torch.cuda.Event()
        ev_trk.record(self.s_trk)
        self.trk_events[k] = ev_trk
        self.inflight.append(_Tick(k, metas, ev_pre, ev_trk, r, spans))
        self.ticks += 1

    def _submit_one(self, fr: Frame):
        """A tick of one frame through the per-stream calls (the same kernels'
        arithmetic, so the same results as a batched tick): no table to pack
        and copy.  With nothing in flight every step goes on the tracking
        stream; otherwise the upload and pyramid go on the preprocessing
        stream, as in a batched tick."""
        import ctypes as C

        from . import ops

        torch, L = self.torch, ops.lib()
        k = self.ticks
        slot = self.slots[fr.sid]
        f = slot.f + 1
        m = slot.m if slot.started else 0
        NF, NP = _Slot.NF, _Slot.NP
        fi, fq, p, q = f % NF, (f - 1) % NF, f % NP, (f - 1) % NP
        sp = slot.spec
        idle = not self.inflight or not self.solo_overlap
        prior = self.trk_events.pop(k - self.depth, None)
        s_pre, h_pre = (self.s_trk, self.h_trk) if idle else (self.s_pre, self.h_pre)
        if prior is not None and not idle:
            s_pre.wait_event(prior)
        slot.upload(fr, f, h_pre)
        self._observe()
        d = ops.OtPyr()
        ops.check(L.ot_pyramid_build(slot.frames[fi].data_ptr(), sp.W, sp.H, sp.W, sp.levels,
                                     slot.ws[fi].data_ptr(), slot.ws[fi].numel(), 0, C.byref(d),
                                     h_pre), "ot_pyramid_build")
        self._observe()
        ev_pre = None
        if not idle:
            ev_pre = torch.cuda.Event()
            ev_pre.record(s_pre)
            self.s_trk.wait_event(ev_pre)
        r = k % (self.depth + 1)
        spans = {}
        if slot.started:
            n = slot.n
            ops.check(L.ot_lk_track_ex(C.byref(slot.pyr[fq].desc), C.byref(slot.pyr[fi].desc),
                                       slot.pts[q].data_ptr(), n, self.cfg.win, sp.levels,
                                       self.cfg.iters, self.cfg.eps, slot.pts[p].data_ptr(),
                                       slot.status.data_ptr(), slot.err.data_ptr(),
                                       C.byref(self.opts), self.h_trk), "ot_lk_track")
            self._observe()
            ops.check(L.ot_box_update(slot.boxes[q].data_ptr(), m, slot.box_id.data_ptr(),
                                      slot.pts[q].data_ptr(), slot.pts[p].data_ptr(),
                                      slot.status.data_ptr(), n, slot.boxes[p].data_ptr(),
                                      slot.count.data_ptr(), self.h_trk), "ot_box_update")
            self._observe()
            if m:
                _copy(self.ring_boxes[r][p][slot.c0:].data_ptr(), slot.boxes[p].data_ptr(),
                      m * 16, _D2H, self.h_trk)
                _copy(self.ring_count[r][slot.c0:].data_ptr(), slot.count.data_ptr(), m * 4,
                      _D2H, self.h_trk)
                spans[p] = (slot.c0, slot.c0 + m)
        self._observe()
        slot.reseed(fr, f, self.h_trk)
        slot.f = f
        ev_trk = torch.cuda.Event()
        ev_trk.record(self.s_trk)
        self.trk_events[k] = ev_trk
        self.inflight.append(_Tick(k, [(fr, slot, f, m)], ev_pre, ev_trk, r, spans))
        self.ticks += 1

    def _collect(self, tk: _Tick, t_done: float) -> list:
        out = []
        hb = [b.numpy() for b in self.ring_boxes[tk.ring]]
        hc = self.ring_count[tk.ring].numpy()
        for fr, slot, f, m in tk.metas:
            par = f % _Slot.NP
            out.append(Result(fr.sid, fr.k, fr.t_arrival, t_done,
                              hb[par][slot.c0:slot.c0 + m].copy(),
                              hc[slot.c0:slot.c0 + m].copy(), tk.idx))
            slot.frames_done += 1
        return out

    def poll(self, now=time.perf_counter) -> list:
        """Results of the ticks that have completed, oldest first (no wait)."""
        out, self.ready = self.ready, []
        while self.inflight:
            tk = self.inflight[0]
            if tk.t_done is None:
                if not tk.ev_trk.query():
                    break
                tk.t_done = now()
            out += self._collect(self.inflight.popleft(), tk.t_done)
        return out

    def wait_until(self, stop, now=time.perf_counter) -> None:
        """Spin until the oldest tick in flight completes (its results are on
        the host from that moment: the time is kept for them) or stop() is
        true."""
        if not self.inflight:
            return
        tk = self.inflight[0]
        while tk.t_done is None:
            if tk.ev_trk.query():
                tk.t_done = now()
                return
            if stop():
                return

    def wait_oldest(self, now=time.perf_counter) -> list:
        """Block until the oldest tick in flight completes; its results."""
        if not self.inflight:
            return []
        tk = self.inflight.popleft()
        if tk.t_done is None:
            tk.ev_trk.synchronize()
            tk.t_done = now()
        return self._collect(tk, tk.t_done)

    def drain(self, now=time.perf_counter) -> list:
        out = []
        while self.inflight:
            out += self.wait_oldest(now)
        return out

    def run_tick(self, frames: list, now=time.perf_counter) -> list:
        """One tick, blocking: submit and wait (results of any earlier ticks
        in flight come first)."""
        out = self.drain(now)
        self.submit(frames, now)
        return out + self.drain(now)


class PlainExecutor:
    """The comparison path: each frame on its own with the per-stream calls
    (ot_pyramid_build, ot_lk_track, ot_box_update), in arrival order, on one
    stream, waiting for each frame's boxes before the next frame starts, with
    the same resident state and the same copies as the served path."""

    def __init__(self, win=21, iters=30, eps=0.01, device="cuda", max_slots=128, m_chunk=64):
        import torch

        from . import ops

        self.torch = torch
        self.device = torch.device(device)
        self.win, self.iters, self.eps = win, iters, eps
        self.arena = _Arena(torch, self.device, max_slots, m_chunk)
        self.slots: dict = {}
        self.stream = torch.cuda.Stream(self.device)
        self.sh = int(self.stream.cuda_stream)
        self.opts = ops.OtLkOpts(ops.OT_DEFAULT_MIN_EIG, None, None, 0, 0, None)
        self.ticks = 0
        torch.cuda.synchronize(self.device)  # the arena's fills precede the stream's work

    def admit(self, spec: StreamSpec):
        self.slots[spec.sid] = _Slot(spec, self.device, self.arena, self.stream)

    def evict(self, sid: int):
        s = self.slots.pop(sid, None)
        if s is not None:
            self.torch.cuda.synchronize(self.device)
            s.release()

    def run_tick(self, frames: list, now=time.perf_counter) -> list:
        import ctypes as C

        from . import ops

        torch, L = self.torch, ops.lib()
        for fr in frames:
            check_frame(fr, self.slots[fr.sid].spec)
        out = []
        a = self.arena
        NF, NP = _Slot.NF, _Slot.NP
        for fr in frames:
            slot = self.slots[fr.sid]
            f = slot.f + 1
            fi, fq = f % NF, (f - 1) % NF
            p, q = f % NP, (f - 1) % NP
            sp = slot.spec
            slot.upload(fr, f, self.sh)
            d = ops.OtPyr()
            ops.check(L.ot_pyramid_build(slot.frames[fi].data_ptr(), sp.W, sp.H, sp.W, sp.levels,
                                         slot.ws[fi].data_ptr(), slot.ws[fi].numel(), 0,
                                         C.byref(d), self.sh), "ot_pyramid_build")
            m = 0
            if slot.started:
                n, m = slot.n, slot.m
                ops.check(L.ot_lk_track_ex(C.byref(slot.pyr[fq].desc), C.byref(slot.pyr[fi].desc),
                                           slot.pts[q].data_ptr(), n, self.win, sp.levels,
                                           self.iters, self.eps, slot.pts[p].data_ptr(),
                                           slot.status.data_ptr(), slot.err.data_ptr(),
                                           C.byref(self.opts), self.sh), "ot_lk_track")
                ops.check(L.ot_box_update(slot.boxes[q].data_ptr(), m, slot.box_id.data_ptr(),
                                          slot.pts[q].data_ptr(), slot.pts[p].data_ptr(),
                                          slot.status.data_ptr(), n, slot.boxes[p].data_ptr(),
                                          slot.count.data_ptr(), self.sh), "ot_box_update")
                _copy(a.host_boxes[p][slot.c0:].data_ptr(), slot.boxes[p].data_ptr(), m * 16,
                      _D2H, self.sh)
                _copy(a.host_count[slot.c0:].data_ptr(), slot.count.data_ptr(), m * 4, _D2H,
                      self.sh)
            slot.reseed(fr, f, self.sh)
            ev = torch.cuda.Event()
            ev.record(self.stream)
            while not ev.query():   # the same host wait as the served path
                pass
            out.append(Result(fr.sid, fr.k, fr.t_arrival, now(),
                              a.host_boxes[p].numpy()[slot.c0:slot.c0 + m].copy(),
                              a.host_count.numpy()[slot.c0:slot.c0 + m].copy(), self.ticks))
            slot.f = f
            slot.frames_done += 1
            self.ticks += 1
        return out


# ----------------------------------------------------------------------------- driver
def make_trace(nstreams: int, duration: float, fps: float, seed: int, rate_scale: float = 1.0):
    """Poisson arrivals per stream (exponential gaps, mean 1/(fps*rate_scale)),
    start offsets U[0, 1/fps).  Returns a sorted list of (t, sid, k)."""
    rng = np.random.default_rng(seed)
    out = []
    lam = fps * rate_scale
    for s in range(nstreams):
        t = rng.uniform(0.0, 1.0 / fps)
        k = 0
        while t < duration:
            out.append((t, s, k))
            t += rng.exponential(1.0 / lam)
            k += 1
    out.sort()
    return out


# the OS wakes a sleeping thread up to this late: waits end in a spin
_SPIN_S = 1e-3


def _wait(clock, dt: float):
    """Wait dt seconds: sleep while more than the OS's wake-up slack remains,
    then spin to the exact time (an arrival is noticed within microseconds,
    not at the next scheduler wake-up)."""
    end = clock() + dt
    if dt > 2 * _SPIN_S:
        time.sleep(dt - _SPIN_S)
    while clock() < end:
        pass


def run_trace(trace, frame_fn, specs, scheduler: Scheduler, executor, clock=None,
              sleep=None, max_wall: float | None = None, batched: bool = True):
    """Drive arrivals against a clock.  `frame_fn(sid, k, t)` returns a Frame.
    With the real clock, arrivals are released when their time has come and,
    while nothing waits, the loop sleeps and then spins to the next arrival;
    with a fake clock, `sleep` advances it.  `batched=False` processes waiting frames one at a time (FIFO over
    all streams).  Returns the list of Results."""
    clock = clock or time.perf_counter
    sleep = sleep or (lambda dt: _wait(clock, dt))
    for sp in specs:
        scheduler.register(sp)
    # Python's cycle collector stops the loop for tens of milliseconds once
    # thousands of results are alive, and every frame queued meanwhile waits
    # that long: it stays off while the loop runs (reference counting still
    # frees everything that is not in a cycle) and runs once afterwards.
    gc_on = gc.isenabled()
    gc.disable()
    try:
        if batched and hasattr(executor, "submit"):
            return _run_trace_pipelined(trace, frame_fn, scheduler, executor, clock, sleep,
                                        max_wall)
        return _run_trace(trace, frame_fn, scheduler, executor, clock, sleep, max_wall, batched)
    finally:
        if gc_on:
            gc.enable()
        gc.collect()


def _run_trace(trace, frame_fn, scheduler, executor, clock, sleep, max_wall, batched):
    t0 = clock()
    i, results = 0, []
    n = len(trace)
    while i < n or scheduler.pending():
        now = clock() - t0
        if max_wall is not None and now > max_wall:
            break
        while i < n and trace[i][0] <= now:
            t, sid, k = trace[i]
            scheduler.arrive(frame_fn(sid, k, t))
            i += 1
        for sid in scheduler.evict_idle(now):
            executor.evict(sid)
        for sid in scheduler.admit():
            executor.admit(scheduler.specs[sid])
        frames = scheduler.next_batch()
        if not batched:
            frames.sort(key=lambda f: f.t_arrival)
            scheduler.requeue(frames[1:])
            frames = frames[:1]
        if frames:
            res = executor.run_tick(frames, now=lambda: clock() - t0)
            results += res
            continue
        # nothing runnable: wait for the next arrival or the next eviction that
        # could free budget for a waiting stream
        wake = [trace[i][0]] if i < n else []
        if scheduler.waiting:
            wake += scheduler.eviction_times(now)
        if not wake:
            break  # frames wait for streams that can never be admitted
        sleep(min(wake) - (clock() - t0) + 1e-6)
    return results


def _run_trace_pipelined(trace, frame_fn, scheduler, executor, clock, sleep, max_wall):
    """The loop for an executor with ticks in flight (submit / poll / busy /
    wait_until): frames that arrive while ticks run are admitted and
    submitted as soon as the executor takes another tick, and results are
    collected as their ticks complete."""
    t0 = clock()
    i, results = 0, []
    n = len(trace)

    def now():
        return clock() - t0

    while i < n or scheduler.pending() or executor.busy():
        t = now()
        if max_wall is not None and t > max_wall:
            break
        while i < n and trace[i][0] <= t:
            ts, sid, k = trace[i]
            scheduler.arrive(frame_fn(sid, k, ts))
            i += 1
        results += executor.poll(now)
        for sid in scheduler.evict_idle(t):
            executor.evict(sid)
        for sid in scheduler.admit():
            executor.admit(scheduler.specs[sid])
        if executor.can_submit():
            frames = scheduler.next_batch()
            if frames:
                executor.submit(frames, now)
                continue
        if executor.busy():
            due = trace[i][0] if i < n else math.inf
            executor.wait_until(lambda: now() >= due, now)
            continue
        wake = [trace[i][0]] if i < n else []
        if scheduler.waiting:
            wake += scheduler.eviction_times(t)
        if not wake:
            break
        sleep(min(wake) - now() + 1e-6)
    results += executor.poll(now)
    results += executor.drain(now)
    return results


def latency_stats(results) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    if len(lat) == 0:
        return {"frames": 0}
    return {"frames": int(len(lat)), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max())}
