"""Batched tick over many independent streams (one frame pair each).

A tick builds every job's new pyramid, tracks every job's points and
updates every job's boxes, one launch per stage (one per pyramid level),
all reading a descriptor table that `ot_batch_pack` writes into pinned host
memory and `ot_batch_run` copies to the device.  Because the launch shapes
depend only on the table capacities, a tick can be captured once as a HIP
graph and replayed with any later table of the same capacities.

`Autotuner` times the schedule knobs of the tracking stage (LDS margin,
one wave per point vs a persistent grid claiming chunks of points) on a
representative tick and caches the fastest per shape bucket in a JSON file.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
from dataclasses import dataclass, asdict, field

from . import ops

__all__ = ["Job", "BatchConfig", "BatchRunner", "Autotuner", "bucket_key"]


@dataclass
class Job:
    """One stream's frame pair: resident previous pyramid, new frame (device),
    workspace for the new pyramid, points/boxes and output buffers (all torch
    CUDA tensors)."""

    prev: "ops.Pyramid"
    next_frame: object
    next_ws: object
    levels: int
    pts: object
    next_pts: object
    status: object
    err: object
    boxes: object
    box_id: object
    out_boxes: object
    out_count: object

    @property
    def n(self) -> int:
        return int(self.pts.shape[0])

    @property
    def m(self) -> int:
        return int(self.boxes.shape[0])


@dataclass
class BatchConfig:
    win: int = 21
    iters: int = 30
    eps: float = 0.01
    min_eig: float = ops.OT_DEFAULT_MIN_EIG
    margin: int = 0
    lk_waves: int = 0          # 0: one wave per point; >0: persistent grid of this many waves
    chunk: int = 1
    lk_wpg: int = 1            # waves per workgroup of the tracking stage (1, 2, 4)
    lk_ppw: int = 1            # points each wave tracks in turn (1, 2, 4)
    max_jobs: int = 64
    max_points: int = 1 << 20
    max_boxes: int = 4096
    max_tiles: int = 1 << 14
    max_levels: int = 5
    exact_grids: bool = False  # eager ticks: launch exactly the packed work

    def to_c(self) -> "ops.OtBatchCfg":
        return ops.OtBatchCfg(self.win, self.iters, self.eps, self.min_eig, self.margin,
                              self.lk_waves, self.chunk, self.max_jobs, self.max_points,
                              self.max_boxes, self.max_tiles, self.max_levels,
                              int(self.exact_grids), self.lk_wpg, self.lk_ppw)

    def schedule(self) -> dict:
        return {"margin": self.margin, "lk_waves": self.lk_waves, "chunk": self.chunk,
                "lk_wpg": self.lk_wpg, "lk_ppw": self.lk_ppw}


def _ptr(t):
    return None if t is None else int(t.data_ptr())


def jobs_from_workloads(workloads: list, device="cuda") -> list:
    """Device-resident jobs for synthetic frame pairs: frame 0's pyramid is
    built (resident), frame 1 and all point/box inputs are uploaded, outputs
    allocated."""
    import numpy as np
    import torch

    dev = torch.device(device)

    def t(x):
        return torch.from_numpy(np.ascontiguousarray(x)).to(dev)

    jobs = []
    for w in workloads:
        H, W = w.frame0.shape
        n, m = w.n, w.boxes.shape[0]
        jobs.append(Job(prev=ops.pyramid_build(t(w.frame0), w.levels), next_frame=t(w.frame1),
                        next_ws=ops.alloc_workspace(W, H, w.levels, dev), levels=w.levels,
                        pts=t(w.pts), next_pts=torch.empty((n, 2), device=dev),
                        status=torch.empty(n, dtype=torch.uint8, device=dev),
                        err=torch.empty(n, device=dev), boxes=t(w.boxes), box_id=t(w.box_id),
                        out_boxes=torch.empty((m, 4), device=dev),
                        out_count=torch.empty(m, dtype=torch.int32, device=dev)))
    return jobs


def _c_jobs(jobs: list):
    """The ot_job array for `jobs` (device pointers only; nothing is copied)."""
    arr = (ops.OtJob * max(1, len(jobs)))()
    for i, j in enumerate(jobs):
        o = arr[i]
        o.prev = j.prev.desc
        o.next_frame = _ptr(j.next_frame)
        o.next_pitch = int(j.next_frame.stride(0))
        o.next_ws = _ptr(j.next_ws)
        o.next_ws_bytes = int(j.next_ws.numel()) if j.next_ws is not None else 0
        o.levels = j.levels
        o.pts, o.n = _ptr(j.pts), j.n
        o.next_pts, o.status, o.err = _ptr(j.next_pts), _ptr(j.status), _ptr(j.err)
        o.boxes, o.m, o.box_id = _ptr(j.boxes), j.m, _ptr(j.box_id)
        o.out_boxes, o.out_count = _ptr(j.out_boxes), _ptr(j.out_count)
    return arr


_E_WORKSPACE = next(k for k, v in ops.ERRORS.items() if v == "OT_E_WORKSPACE")


def fit_capacities(cfg: BatchConfig, jobs: list) -> BatchConfig:
    """cfg with the smallest capacities `jobs` fit: jobs, points and boxes
    are their totals, and the pyramid tiles are found by bisection with
    ot_batch_pack (host only), which refuses a table whose fused pyramid
    stages need more tiles than max_tiles.  A graph captured for a bucket of
    ticks with these capacities launches no idle workgroups for them."""
    import dataclasses

    import torch

    arr = _c_jobs(jobs)
    base = dataclasses.replace(cfg, max_jobs=max(1, len(jobs)),
                               max_points=max(1, sum(j.n for j in jobs)),
                               max_boxes=max(1, sum(j.m for j in jobs)))

    def fits(tiles: int) -> bool:
        c = dataclasses.replace(base, max_tiles=tiles).to_c()
        nb = int(ops.lib().ot_batch_table_bytes(C.byref(c)))
        host = torch.empty(nb, dtype=torch.uint8)
        e = int(ops.lib().ot_batch_pack(arr, len(jobs), C.byref(c), int(host.data_ptr()), nb, None))
        if e not in (0, _E_WORKSPACE):
            ops.check(e, "ot_batch_pack")
        return e == 0

    hi = max(1, cfg.max_tiles)
    if not fits(hi):
        raise ValueError("the jobs need more pyramid tiles than cfg.max_tiles")
    lo = 0  # fits(lo) is false for any non-empty pyramid stage; hi fits
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if fits(mid):
            hi = mid
        else:
            lo = mid
    return dataclasses.replace(base, max_tiles=hi)


class BatchRunner:
    """Owns the pinned host table and the device table for one capacity."""

    def __init__(self, cfg: BatchConfig, device="cuda", tables: int = 2):
        import torch

        self.torch = torch
        self.cfg = cfg
        self.ccfg = cfg.to_c()
        nb = int(ops.lib().ot_batch_table_bytes(C.byref(self.ccfg)))
        if nb == 0:
            raise ValueError("invalid batch configuration")
        self.table_bytes = nb
        # several host tables so the next tick can be packed while the last copy is pending
        self.host = [torch.empty(nb, dtype=torch.uint8, pin_memory=True) for _ in range(tables)]
        self.dev = torch.empty(nb, dtype=torch.uint8, device=device)
        self.events = [None] * tables
        self.cur = 0
        self.next_pyrs = []

    def pack(self, jobs: list, table: int | None = None) -> list:
        """Write the table for `jobs`; returns each job's new pyramid (ops.Pyramid)."""
        t = self.cur if table is None else table
        ev = self.events[t]
        if ev is not None:
            ev.synchronize()  # the copy that last read this host table has executed
        arr = _c_jobs(jobs)
        nxt = (ops.OtPyr * max(1, len(jobs)))()
        ops.check(ops.lib().ot_batch_pack(arr, len(jobs), C.byref(self.ccfg),
                                          int(self.host[t].data_ptr()), self.table_bytes, nxt),
                  "ot_batch_pack")
        self.cur = t
        self.next_pyrs = [ops.Pyramid(j.next_frame, j.next_ws, nxt[i]) for i, j in enumerate(jobs)]
        return self.next_pyrs

    def run(self, stream=None, table: int | None = None):
        """Copy the packed table to the device and launch the stages."""
        torch = self.torch
        t = self.cur if table is None else table
        s = stream if stream is not None else torch.cuda.current_stream()
        ops.check(ops.lib().ot_batch_run(int(self.host[t].data_ptr()), int(self.dev.data_ptr()),
                                         self.table_bytes, C.byref(self.ccfg), int(s.cuda_stream)),
                  "ot_batch_run")
        ev = torch.cuda.Event()
        ev.record(s)
        self.events[t] = ev
        self.cur = (t + 1) % len(self.host)

    def capture(self, table: int = 0):
        """A HIP graph of one tick reading host table `table` (replay after
        re-packing that table with the same capacities)."""
        torch = self.torch
        if self.cfg.exact_grids:
            raise ValueError("a captured tick needs capacity-sized grids (exact_grids=False)")
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=s):
            ops.check(ops.lib().ot_batch_run(int(self.host[table].data_ptr()),
                                             int(self.dev.data_ptr()), self.table_bytes,
                                             C.byref(self.ccfg), int(s.cuda_stream)),
                      "ot_batch_run")
        torch.cuda.synchronize()
        return g


_DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def default_schedule(key: str, grads: bool | None = None) -> dict:
    """Tuned schedule for a shape bucket from the packaged cache (nearest
    point bucket), else one wave per point with the default margin.  For the
    single-call tracker, `grads` False/True restricts the choice to gradients
    computed in the tracker / read from materialized planes."""
    if os.path.exists(_DEFAULT_CACHE):
        with open(_DEFAULT_CACHE) as f:
            cache = json.load(f)

        def pick(rec):
            if grads is None or "all" not in rec:
                return dict(rec["schedule"])
            ok = [r for r in rec["all"] if bool(r.get("grads", False)) == grads]
            if not ok:
                return dict(rec["schedule"])
            best = min(ok, key=lambda r: r["ms"])
            return {k: v for k, v in best.items() if k != "ms"}

        if key in cache:
            return pick(cache[key])
        single = key.startswith("single_")
        cands = [k for k in cache if k.startswith("single_") == single]
        if cands:
            def pts(k):
                return int(k.split("_")[-2][1:])
            want = pts(key)
            best = min(cands, key=lambda k: abs(math.log2(pts(k)) - math.log2(want)))
            return pick(cache[best])
    return ({"margin": 0} if key.startswith("single_") else
            {"margin": 0, "lk_waves": 0, "chunk": 1, "lk_wpg": 1, "lk_ppw": 1})


def bucket_key(jobs: list) -> str:
    """Shape bucket of a tick: total points (power-of-two bucket) and the
    largest level count."""
    pts = sum(j.n for j in jobs)
    return f"p{1 << max(0, math.ceil(math.log2(max(pts, 1))))}_L{max(j.levels for j in jobs)}"


def schedule_space() -> list:
    """Tracking schedules of the batched tick: LDS margin x {waves per
    workgroup x points per wave, one point per wave each, or a persistent
    grid claiming chunks of points}.  Several waves or points per workgroup
    exist for the 21 x 21 window at margins 4 and 6."""
    out = []
    for m in (2, 3, 4, 6):
        shapes = [(1, 1)]
        if m in (4, 6):
            shapes = [(w, p) for w in (1, 2, 4) for p in (1, 2, 4)]
        for (w, p) in shapes:
            out.append({"margin": m, "lk_waves": 0, "chunk": 1, "lk_wpg": w, "lk_ppw": p})
        for (w, c) in ((4096, 1), (4096, 4), (8192, 2)):
            out.append({"margin": m, "lk_waves": w, "chunk": c, "lk_wpg": 1, "lk_ppw": 1})
    return out


@dataclass
class Autotuner:
    """Times candidate tracking schedules on a tick and caches the best."""

    path: str | None = None
    candidates: list = field(default_factory=schedule_space)
    cache: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.path and os.path.exists(self.path):
            with open(self.path) as f:
                self.cache = json.load(f)

    def best(self, key: str):
        return self.cache.get(key, {}).get("schedule")

    def tune(self, jobs: list, base: BatchConfig, reps: int = 10, warmup: int = 3) -> dict:
        """Try every candidate on `jobs`; returns {schedule, ms, all}."""
        import torch

        key = bucket_key(jobs)
        results = []
        for cand in self.candidates:
            cfg = BatchConfig(**{**asdict(base), **cand})
            runner = BatchRunner(cfg, device=jobs[0].pts.device, tables=1)
            runner.pack(jobs, table=0)
            g = runner.capture(0)
            for _ in range(warmup):
                g.replay()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                g.replay()
            e1.record()
            torch.cuda.synchronize()
            results.append((e0.elapsed_time(e1) / reps, cand))
            del g, runner
        results.sort(key=lambda r: r[0])
        rec = {"schedule": results[0][1], "ms": results[0][0],
               "all": [{"ms": ms, **c} for ms, c in results]}
        self.cache[key] = rec
        if self.path:
            os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
            with open(self.path, "w") as f:
                json.dump(self.cache, f, indent=1)
        return rec
