"""Continuous-batching serving loop for many video streams on one GPU.

Frames arrive per stream at their own times.  The scheduler admits a stream
when its resident state fits the HBM budget (otherwise it waits in FIFO
order), and every tick batches the oldest waiting frame of every admitted
stream into one batched launch (new pyramid, tracking, box update; see
`batch.py`).  Frames that arrive while a tick runs join the next tick.  A
stream's previous pyramid, points and boxes stay resident between frames:
each frame builds one pyramid and the two pyramid workspaces swap roles.
Every `reseed_every`-th frame replaces the stream's boxes and points with
synthetic "detections".  Streams silent for `evict_after` seconds are evicted
and their memory returned to the budget.

`Scheduler` is pure Python (no GPU) so admission, batching order and
eviction are testable with a fake clock and a fake executor; `GpuExecutor`
runs ticks on the device through the C ABI, and `PlainExecutor` processes
the same frames one at a time with the per-stream calls for comparison.
"""
from __future__ import annotations

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
class _Slot:
    """Resident device state of one stream."""

    def __init__(self, spec: StreamSpec, device):
        import torch

        from . import ops

        self.spec = spec
        H, W, L = spec.H, spec.W, spec.levels
        self.frames = [torch.empty((H, W), dtype=torch.uint8, device=device) for _ in range(2)]
        self.ws = [ops.alloc_workspace(W, H, L, device) for _ in range(2)]
        n, m = spec.n_max, spec.m_max
        self.pts = [torch.zeros((n, 2), dtype=torch.float32, device=device) for _ in range(2)]
        self.status = torch.zeros(n, dtype=torch.uint8, device=device)
        self.err = torch.zeros(n, dtype=torch.float32, device=device)
        self.box_id = torch.full((n,), -1, dtype=torch.int32, device=device)
        self.boxes = [torch.zeros((m, 4), dtype=torch.float32, device=device) for _ in range(2)]
        self.count = torch.zeros(m, dtype=torch.int32, device=device)
        self.cur = 0            # index of the frame / pyramid / points / boxes of the last frame
        self.pyr = None         # ops.Pyramid of the last frame
        self.n = 0
        self.m = 0
        self.frames_done = 0


class GpuExecutor:
    """Runs a tick of frames (at most one per stream) as one batched launch."""

    def __init__(self, win=21, iters=30, eps=0.01, max_jobs=64, max_points=1 << 21,
                 max_boxes=4096, max_levels=5, schedule=None, device="cuda"):
        import torch

        from . import batch

        self.torch = torch
        self.device = torch.device(device)
        sched = schedule or {}
        self.cfg = batch.BatchConfig(win=win, iters=iters, eps=eps, max_jobs=max_jobs,
                                     max_points=max_points, max_boxes=max_boxes,
                                     max_tiles=1 << 15, max_levels=max_levels, **sched)
        self.runner = batch.BatchRunner(self.cfg, device=self.device, tables=2)
        self.slots: dict = {}
        self.stream = torch.cuda.Stream()
        self.host_boxes = torch.empty((max_boxes, 4), dtype=torch.float32, pin_memory=True)
        self.host_count = torch.empty(max_boxes, dtype=torch.int32, pin_memory=True)
        self.dev_boxes = torch.empty((max_boxes, 4), dtype=torch.float32, device=self.device)
        self.dev_count = torch.empty(max_boxes, dtype=torch.int32, device=self.device)
        self.ticks = 0

    def admit(self, spec: StreamSpec):
        self.slots[spec.sid] = _Slot(spec, self.device)

    def evict(self, sid: int):
        self.slots.pop(sid, None)

    @staticmethod
    def _upload(torch, slot, fr: Frame, nxt: int):
        src = fr.pixels if isinstance(fr.pixels, torch.Tensor) else torch.from_numpy(fr.pixels)
        slot.frames[nxt].copy_(src, non_blocking=True)

    @staticmethod
    def _reseed(torch, slot, fr: Frame, dst: int):
        """Detections at this frame replace the points and boxes tracked from it
        (after the frame's own pair has been processed)."""
        if fr.reseed is None:
            return
        p, bid, bx = fr.reseed
        n, m = len(p), len(bx)
        if n > slot.spec.n_max or m > slot.spec.m_max:
            raise ValueError("detections exceed the stream's capacity")
        slot.pts[dst][:n].copy_(torch.from_numpy(np.ascontiguousarray(p)), non_blocking=True)
        slot.box_id[:n].copy_(torch.from_numpy(np.ascontiguousarray(bid)), non_blocking=True)
        slot.boxes[dst][:m].copy_(torch.from_numpy(np.ascontiguousarray(bx)), non_blocking=True)
        slot.n, slot.m = n, m

    def run_tick(self, frames: list, now=time.perf_counter) -> list:
        torch = self.torch
        from . import batch, ops

        jobs, metas = [], []
        with torch.cuda.stream(self.stream):
            for fr in frames:
                slot = self.slots[fr.sid]
                nxt = 1 - slot.cur
                self._upload(torch, slot, fr, nxt)
                first = slot.pyr is None
                n = 0 if first else slot.n
                m = 0 if first else slot.m
                prev = slot.pyr if not first else ops.pyramid_layout(
                    slot.frames[nxt], slot.spec.levels, slot.ws[nxt])
                jobs.append(batch.Job(
                    prev=prev, next_frame=slot.frames[nxt], next_ws=slot.ws[nxt],
                    levels=slot.spec.levels, pts=slot.pts[slot.cur][:n],
                    next_pts=slot.pts[nxt][:n], status=slot.status[:n], err=slot.err[:n],
                    boxes=slot.boxes[slot.cur][:m], box_id=slot.box_id[:n],
                    out_boxes=slot.boxes[nxt][:m], out_count=slot.count[:m]))
                metas.append((fr, slot, nxt, m))
            pyrs = self.runner.pack(jobs)
            self.runner.run(self.stream)
            # gather every stream's outputs into one buffer for a single copy back
            off = 0
            for (fr, slot, nxt, m), _ in zip(metas, jobs):
                if m:
                    self.dev_boxes[off:off + m].copy_(slot.boxes[nxt][:m])
                    self.dev_count[off:off + m].copy_(slot.count[:m])
                off += m
            tot = off
            for fr, slot, nxt, m in metas:
                self._reseed(torch, slot, fr, nxt)
            if tot:
                self.host_boxes[:tot].copy_(self.dev_boxes[:tot], non_blocking=True)
                self.host_count[:tot].copy_(self.dev_count[:tot], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        ev.synchronize()
        t = now()
        out, off = [], 0
        for (fr, slot, nxt, m), pyr in zip(metas, pyrs):
            slot.pyr = pyr
            slot.cur = nxt
            slot.frames_done += 1
            out.append(Result(fr.sid, fr.k, fr.t_arrival, t,
                              self.host_boxes[off:off + m].numpy().copy(),
                              self.host_count[off:off + m].numpy().copy(), self.ticks))
            off += m
        self.ticks += 1
        return out


class PlainExecutor:
    """The comparison path: each frame on its own, with the per-stream calls
    (ot_pyramid_build, ot_lk_track, ot_box_update), in arrival order."""

    def __init__(self, win=21, iters=30, eps=0.01, device="cuda"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.win, self.iters, self.eps = win, iters, eps
        self.slots: dict = {}
        self.stream = torch.cuda.Stream()
        self.ticks = 0

    def admit(self, spec: StreamSpec):
        self.slots[spec.sid] = _Slot(spec, self.device)

    def evict(self, sid: int):
        self.slots.pop(sid, None)

    def run_tick(self, frames: list, now=time.perf_counter) -> list:
        torch = self.torch
        from . import ops

        out = []
        for fr in frames:
            slot = self.slots[fr.sid]
            nxt = 1 - slot.cur
            with torch.cuda.stream(self.stream):
                GpuExecutor._upload(torch, slot, fr, nxt)
                Q = ops.pyramid_build(slot.frames[nxt], slot.spec.levels, ws=slot.ws[nxt],
                                      stream=self.stream)
                m = 0
                if slot.pyr is not None:
                    n, m = slot.n, slot.m
                    ops.lk_track(slot.pyr, Q, slot.pts[slot.cur][:n], win=self.win,
                                 levels=slot.spec.levels, iters=self.iters, eps=self.eps,
                                 out=(slot.pts[nxt][:n], slot.status[:n], slot.err[:n]),
                                 stream=self.stream)
                    ops.box_update(slot.boxes[slot.cur][:m], slot.box_id[:n],
                                   slot.pts[slot.cur][:n], slot.pts[nxt][:n], slot.status[:n],
                                   out=(slot.boxes[nxt][:m], slot.count[:m]), stream=self.stream)
                hb = slot.boxes[nxt][:m].to("cpu", non_blocking=True)
                hc = slot.count[:m].to("cpu", non_blocking=True)
                GpuExecutor._reseed(torch, slot, fr, nxt)
                ev = torch.cuda.Event()
                ev.record(self.stream)
            ev.synchronize()
            slot.pyr = Q
            slot.cur = nxt
            out.append(Result(fr.sid, fr.k, fr.t_arrival, now(), hb.numpy().copy(),
                              hc.numpy().copy(), self.ticks))
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
