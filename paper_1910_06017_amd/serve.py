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
import heapq
import math
import time
from collections import deque
from dataclasses import dataclass, field

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

    def __init__(self, budget: int, max_jobs: int, max_points: int, evict_after: float = 2.0,
                 footprint=stream_footprint):
        self.budget, self.max_jobs, self.max_points = budget, max_jobs, max_points
        self.evict_after = evict_after
        self.footprint = footprint
        self.specs: dict = {}
        self.admitted: dict = {}     # sid -> bytes
        self.waiting: deque = deque()  # sids waiting for admission, FIFO
        self.queues: dict = {}       # sid -> deque of frames
        self.last_seen: dict = {}
        self.used = 0
        self.evicted: list = []
        self.rejected: list = []

    def register(self, spec: StreamSpec):
        self.specs[spec.sid] = spec
        self.queues.setdefault(spec.sid, deque())

    def arrive(self, fr: Frame):
        q = self.queues[fr.sid]
        q.append(fr)
        self.last_seen[fr.sid] = fr.t_arrival
        if fr.sid not in self.admitted and fr.sid not in self.waiting:
            fp = self.footprint(self.specs[fr.sid])
            if fp > self.budget:
                self.rejected.append(fr.sid)   # can never fit
                q.clear()
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
        gone = []
        for sid in list(self.admitted):
            if not self.queues[sid] and now - self.last_seen.get(sid, now) > self.evict_after:
                self.used -= self.admitted.pop(sid)
                gone.append(sid)
        self.evicted += gone
        return gone

    def next_batch(self) -> list:
        """Oldest waiting frame of each admitted stream (oldest first), within
        the per-tick job and point capacities."""
        cands = [(q[0].t_arrival, sid) for sid, q in self.queues.items()
                 if q and sid in self.admitted]
        cands.sort()
        batch, pts = [], 0
        for _, sid in cands:
            n = self.specs[sid].n_max
            if len(batch) >= self.max_jobs or pts + n > self.max_points:
                break
            batch.append(self.queues[sid].popleft())
            pts += n
        return batch

    def pending(self) -> int:
        return sum(len(q) for q in self.queues.values())


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
    """Resident device state of one stream: two frames, two pyramid
    workspaces, two point buffers and two box chunks (one per frame parity),
    plus the C job descriptors of both parities, built once."""

    def __init__(self, spec: StreamSpec, device, arena: _Arena):
        import ctypes as C

        import torch

        from . import ops

        if spec.m_max > arena.m_chunk:
            raise ValueError(f"stream {spec.sid}: {spec.m_max} boxes > {arena.m_chunk} per stream")
        self.spec = spec
        H, W, L = spec.H, spec.W, spec.levels
        self.frames = [torch.empty((H, W), dtype=torch.uint8, device=device) for _ in range(2)]
        self.ws = [ops.alloc_workspace(W, H, L, device) for _ in range(2)]
        n = max(1, spec.n_max)
        self.pts = [torch.zeros((n, 2), dtype=torch.float32, device=device) for _ in range(2)]
        self.status = torch.zeros(n, dtype=torch.uint8, device=device)
        self.err = torch.zeros(n, dtype=torch.float32, device=device)
        self.box_id = torch.full((n,), -1, dtype=torch.int32, device=device)
        self.arena = arena
        self.chunk = arena.take()
        c0 = self.chunk * arena.m_chunk
        self.c0 = c0
        self.boxes = [arena.dev_boxes[p][c0:c0 + arena.m_chunk] for p in range(2)]
        self.count = arena.dev_count[c0:c0 + arena.m_chunk]
        self.pyr = [ops.pyramid_layout(self.frames[p], L, self.ws[p]) for p in range(2)]
        # job[p]: the frame just uploaded is in parity p, the previous one in 1-p
        self.job = []
        for p in range(2):
            j = ops.OtJob()
            q = 1 - p
            j.prev = self.pyr[q].desc
            j.next_frame = self.frames[p].data_ptr()
            j.next_pitch = W
            j.next_ws = self.ws[p].data_ptr()
            j.next_ws_bytes = self.ws[p].numel()
            j.levels = L
            j.pts, j.next_pts = self.pts[q].data_ptr(), self.pts[p].data_ptr()
            j.status, j.err = self.status.data_ptr(), self.err.data_ptr()
            j.boxes, j.out_boxes = self.boxes[q].data_ptr(), self.boxes[p].data_ptr()
            j.box_id, j.out_count = self.box_id.data_ptr(), self.count.data_ptr()
            self.job.append(j)
        self.cur = 0        # parity of the last frame
        self.started = False
        self.n = 0
        self.m = 0
        self.frames_done = 0
        self._c = C

    def release(self):
        self.arena.give(self.chunk)

    def upload(self, fr: Frame, p: int, stream: int):
        px = fr.pixels
        if hasattr(px, "data_ptr"):
            _copy(self.frames[p].data_ptr(), px.data_ptr(), px.numel(), _H2D, stream)
        else:
            a = np.ascontiguousarray(px, np.uint8)
            _copy(self.frames[p].data_ptr(), a.ctypes.data, a.nbytes, _H2D, stream)

    def reseed(self, fr: Frame, p: int, stream: int):
        """Detections at this frame replace the points and boxes tracked from
        it, after the frame's own pair has been processed."""
        if fr.reseed is None:
            return
        pts, bid, bx = (np.ascontiguousarray(a) for a in fr.reseed)
        n, m = len(pts), len(bx)
        if n > self.spec.n_max or m > self.spec.m_max:
            raise ValueError("detections exceed the stream's capacity")
        pts = pts.astype(np.float32, copy=False)
        bid = bid.astype(np.int32, copy=False)
        bx = bx.astype(np.float32, copy=False)
        # pageable sources: the runtime stages them before the call returns
        _copy(self.pts[p].data_ptr(), pts.ctypes.data, pts.nbytes, _H2D, stream)
        _copy(self.box_id.data_ptr(), bid.ctypes.data, bid.nbytes, _H2D, stream)
        _copy(self.boxes[p].data_ptr(), bx.ctypes.data, bx.nbytes, _H2D, stream)
        self.n, self.m = n, m

    def job_for(self, p: int):
        """C job for the frame in parity p (no points or boxes on the first frame)."""
        j = self.job[p]
        if not self.started:
            j.prev = self.pyr[p].desc   # any valid descriptor: nothing is tracked
            j.n = j.m = 0
        else:
            j.prev = self.pyr[1 - p].desc
            j.n, j.m = self.n, self.m
        return j


class GpuExecutor:
    """Runs a tick of frames (at most one per stream) as one batched launch:
    frame uploads, the table copy and the pyramid, tracking and box stages
    (grids sized to the packed work), one copy back of every result, all on
    one stream."""

    def __init__(self, win=21, iters=30, eps=0.01, max_jobs=64, max_points=1 << 21,
                 max_boxes=4096, max_levels=5, schedule=None, device="cuda", max_slots=128,
                 m_chunk=64):
        import torch

        from . import batch

        self.torch = torch
        self.device = torch.device(device)
        sched = schedule or {}
        self.cfg = batch.BatchConfig(win=win, iters=iters, eps=eps, max_jobs=max_jobs,
                                     max_points=max_points, max_boxes=max_boxes,
                                     max_tiles=1 << 15, max_levels=max_levels, exact_grids=True,
                                     **sched)
        self.runner = batch.BatchRunner(self.cfg, device=self.device, tables=1)
        self.arena = _Arena(torch, self.device, max_slots, m_chunk)
        self.slots: dict = {}
        self.stream = torch.cuda.Stream(self.device)
        self.sh = int(self.stream.cuda_stream)
        self.ticks = 0

    def admit(self, spec: StreamSpec):
        self.slots[spec.sid] = _Slot(spec, self.device, self.arena)

    def evict(self, sid: int):
        s = self.slots.pop(sid, None)
        if s is not None:
            self.torch.cuda.synchronize(self.device)
            s.release()

    def _launch(self, jobs):
        import ctypes as C

        from . import ops

        arr = (ops.OtJob * max(1, len(jobs)))()
        for i, j in enumerate(jobs):
            C.memmove(C.byref(arr, i * C.sizeof(ops.OtJob)), C.byref(j), C.sizeof(ops.OtJob))
        ops.check(ops.lib().ot_batch_pack(arr, len(jobs), C.byref(self.runner.ccfg),
                                          int(self.runner.host[0].data_ptr()),
                                          self.runner.table_bytes, None), "ot_batch_pack")
        # launches sized from the packed totals (a graph would need capacity grids)
        ops.check(ops.lib().ot_batch_run(int(self.runner.host[0].data_ptr()),
                                         int(self.runner.dev.data_ptr()), self.runner.table_bytes,
                                         C.byref(self.runner.ccfg), self.sh), "ot_batch_run")

    def run_tick(self, frames: list, now=time.perf_counter) -> list:
        torch = self.torch
        metas, jobs = [], []
        for fr in frames:
            slot = self.slots[fr.sid]
            p = 1 - slot.cur
            slot.upload(fr, p, self.sh)
            jobs.append(slot.job_for(p))
            metas.append((fr, slot, p, slot.m if slot.started else 0))
        self._launch(jobs)
        a = self.arena
        for par in (0, 1):
            if any(p == par for _, _, p, m in metas if m):
                _copy(a.host_boxes[par].data_ptr(), a.dev_boxes[par].data_ptr(),
                      a.dev_boxes[par].numel() * 4, _D2H, self.sh)
        _copy(a.host_count.data_ptr(), a.dev_count.data_ptr(), a.dev_count.numel() * 4, _D2H,
              self.sh)
        for fr, slot, p, m in metas:
            slot.reseed(fr, p, self.sh)
        ev = torch.cuda.Event()
        ev.record(self.stream)
        ev.synchronize()
        t = now()
        out = []
        hb = [b.numpy() for b in a.host_boxes]
        hc = a.host_count.numpy()
        for fr, slot, p, m in metas:
            out.append(Result(fr.sid, fr.k, fr.t_arrival, t, hb[p][slot.c0:slot.c0 + m].copy(),
                              hc[slot.c0:slot.c0 + m].copy(), self.ticks))
            slot.cur = p
            slot.started = True
            slot.frames_done += 1
        self.ticks += 1
        return out


class PlainExecutor:
    """The comparison path: each frame on its own with the per-stream calls
    (ot_pyramid_build, ot_lk_track, ot_box_update), in arrival order, with the
    same resident state and the same copies as the served path."""

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
        self.opts = ops.OtLkOpts(ops.OT_DEFAULT_MIN_EIG, None, None, 0)
        self.ticks = 0

    def admit(self, spec: StreamSpec):
        self.slots[spec.sid] = _Slot(spec, self.device, self.arena)

    def evict(self, sid: int):
        s = self.slots.pop(sid, None)
        if s is not None:
            self.torch.cuda.synchronize(self.device)
            s.release()

    def run_tick(self, frames: list, now=time.perf_counter) -> list:
        import ctypes as C

        from . import ops

        torch, L = self.torch, ops.lib()
        out = []
        a = self.arena
        for fr in frames:
            slot = self.slots[fr.sid]
            p, q = 1 - slot.cur, slot.cur
            sp = slot.spec
            slot.upload(fr, p, self.sh)
            d = ops.OtPyr()
            ops.check(L.ot_pyramid_build(slot.frames[p].data_ptr(), sp.W, sp.H, sp.W, sp.levels,
                                         slot.ws[p].data_ptr(), slot.ws[p].numel(), 0,
                                         C.byref(d), self.sh), "ot_pyramid_build")
            m = 0
            if slot.started:
                n, m = slot.n, slot.m
                ops.check(L.ot_lk_track_ex(C.byref(slot.pyr[q].desc), C.byref(slot.pyr[p].desc),
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
            slot.reseed(fr, p, self.sh)
            ev = torch.cuda.Event()
            ev.record(self.stream)
            ev.synchronize()
            out.append(Result(fr.sid, fr.k, fr.t_arrival, now(),
                              a.host_boxes[p].numpy()[slot.c0:slot.c0 + m].copy(),
                              a.host_count.numpy()[slot.c0:slot.c0 + m].copy(), self.ticks))
            slot.cur = p
            slot.started = True
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


def run_trace(trace, frame_fn, specs, scheduler: Scheduler, executor, clock=None,
              sleep=None, max_wall: float | None = None, batched: bool = True):
    """Drive arrivals against a clock.  `frame_fn(sid, k, t)` returns a Frame.
    With the real clock, arrivals are released when their time has come and
    the loop sleeps while nothing waits; with a fake clock, `sleep` advances
    it.  `batched=False` processes waiting frames one at a time (FIFO over
    all streams).  Returns the list of Results."""
    clock = clock or time.perf_counter
    sleep = sleep or (lambda dt: time.sleep(max(0.0, dt)))
    for sp in specs:
        scheduler.register(sp)
    # Python's cycle collector stops the loop for tens of milliseconds once
    # thousands of results are alive, and every frame queued meanwhile waits
    # that long: it stays off while the loop runs (reference counting still
    # frees everything that is not in a cycle) and runs once afterwards.
    gc_on = gc.isenabled()
    gc.disable()
    try:
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
            for f in frames[1:]:
                scheduler.queues[f.sid].appendleft(f)
            frames = frames[:1]
        if frames:
            res = executor.run_tick(frames, now=lambda: clock() - t0)
            results += res
            continue
        # nothing runnable: wait for the next arrival or the next eviction that
        # could free budget for a waiting stream
        wake = [trace[i][0]] if i < n else []
        if scheduler.waiting:
            wake += [scheduler.last_seen.get(sid, now) + scheduler.evict_after
                     for sid in scheduler.admitted if not scheduler.queues[sid]]
        if not wake:
            break  # frames wait for streams that can never be admitted
        sleep(min(wake) - (clock() - t0) + 1e-4)
    return results


def latency_stats(results) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    if len(lat) == 0:
        return {"frames": 0}
    return {"frames": int(len(lat)), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max())}
