"""Serving scheduler on the CPU: admission by HBM budget, continuous batching,
eviction of silent streams, capacities, plain FIFO mode -- with a fake clock
and a fake executor (no GPU, no kernels)."""
import numpy as np
import pytest

from paper_1910_06017_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Records ticks; each tick takes `tick_s` of fake time."""

    def __init__(self, clock, tick_s=0.004, per_frame_s=0.0):
        self.clock, self.tick_s, self.per_frame_s = clock, tick_s, per_frame_s
        self.ticks, self.admitted, self.evicted = [], [], []
        self.live = set()

    def admit(self, spec):
        self.admitted.append(spec.sid)
        self.live.add(spec.sid)

    def evict(self, sid):
        self.evicted.append(sid)
        self.live.discard(sid)

    def run_tick(self, frames, now):
        assert all(f.sid in self.live for f in frames)
        self.ticks.append([(f.sid, f.k, f.t_arrival) for f in frames])
        self.clock.t += self.tick_s + self.per_frame_s * len(frames)
        t = now()
        return [serve.Result(f.sid, f.k, f.t_arrival, t, np.zeros((0, 4), np.float32),
                             np.zeros(0, np.int32)) for f in frames]


def spec(sid, W=64, H=48, n=100, m=4):
    return serve.StreamSpec(sid, W, H, 3, n, m)


def frame_fn(sid, k, t):
    return serve.Frame(sid, k, t, None)


def fp_const(nbytes):
    return lambda sp: nbytes


def test_batches_one_frame_per_stream_in_order():
    clock = FakeClock()
    ex = FakeExecutor(clock, tick_s=0.01)
    sch = serve.Scheduler(budget=10**9, max_jobs=64, max_points=10**6, footprint=fp_const(10))
    trace = serve.make_trace(8, 1.0, 25.0, seed=1)
    res = serve.run_trace(trace, frame_fn, [spec(s) for s in range(8)], sch, ex, clock=clock,
                          sleep=clock.sleep)
    assert len(res) == len(trace)
    for tick in ex.ticks:
        sids = [s for s, _, _ in tick]
        assert len(sids) == len(set(sids))          # at most one frame per stream per tick
    last = {}
    for tick in ex.ticks:
        for s, k, _ in tick:
            assert k == last.get(s, -1) + 1         # each stream's frames in order
            last[s] = k
    assert all(r.latency >= 0 for r in res)


def test_frames_arriving_during_a_tick_join_the_next():
    clock = FakeClock()
    ex = FakeExecutor(clock, tick_s=0.05)
    sch = serve.Scheduler(budget=10**9, max_jobs=64, max_points=10**6, footprint=fp_const(10))
    trace = [(0.0, 0, 0), (0.01, 1, 0), (0.02, 2, 0), (0.06, 3, 0)]
    serve.run_trace(trace, frame_fn, [spec(s) for s in range(4)], sch, ex, clock=clock,
                    sleep=clock.sleep)
    assert [len(t) for t in ex.ticks] == [1, 2, 1]
    assert [s for s, _, _ in ex.ticks[1]] == [1, 2]


def test_admission_waits_for_budget_and_evicts_silent_streams():
    clock = FakeClock()
    ex = FakeExecutor(clock, tick_s=0.001)
    sch = serve.Scheduler(budget=250, max_jobs=64, max_points=10**6, evict_after=0.2,
                          footprint=fp_const(100))
    # streams 0 and 1 send two frames then stop; stream 2 starts at 0.05
    trace = [(0.0, 0, 0), (0.0, 1, 0), (0.05, 2, 0), (0.06, 0, 1), (0.07, 1, 1), (0.1, 2, 1),
             (0.5, 2, 2)]
    res = serve.run_trace(trace, frame_fn, [spec(s) for s in range(3)], sch, ex, clock=clock,
                          sleep=clock.sleep)
    assert len(res) == len(trace)
    assert ex.admitted[:2] == [0, 1]
    assert ex.admitted[2] == 2
    # stream 2 could only be admitted after 0 and 1 went silent and were evicted
    first2 = min(r.t_done for r in res if r.sid == 2)
    assert first2 > 0.06 + 0.2
    assert set(sch.evicted) >= {0, 1}
    assert sch.used == 100 * len(sch.admitted)


def test_stream_larger_than_budget_is_rejected():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    sch = serve.Scheduler(budget=50, max_jobs=64, max_points=10**6, footprint=fp_const(100))
    res = serve.run_trace([(0.0, 0, 0), (0.01, 0, 1)], frame_fn, [spec(0)], sch, ex, clock=clock,
                          sleep=clock.sleep)
    assert res == [] and sch.rejected


def test_tick_capacities():
    clock = FakeClock()
    ex = FakeExecutor(clock, tick_s=0.2)
    sch = serve.Scheduler(budget=10**9, max_jobs=3, max_points=250, footprint=fp_const(1))
    trace = [(0.0, s, 0) for s in range(7)]
    serve.run_trace(trace, frame_fn, [spec(s, n=100) for s in range(7)], sch, ex, clock=clock,
                    sleep=clock.sleep)
    assert max(len(t) for t in ex.ticks) <= 2        # 250 points -> two 100-point streams
    assert sum(len(t) for t in ex.ticks) == 7


def test_plain_mode_is_fifo_one_frame_at_a_time():
    clock = FakeClock()
    ex = FakeExecutor(clock, tick_s=0.003)
    sch = serve.Scheduler(budget=10**9, max_jobs=64, max_points=10**6, footprint=fp_const(1))
    trace = serve.make_trace(5, 0.5, 25.0, seed=3)
    res = serve.run_trace(trace, frame_fn, [spec(s) for s in range(5)], sch, ex, clock=clock,
                          sleep=clock.sleep, batched=False)
    assert all(len(t) == 1 for t in ex.ticks)
    arr = [t[0][2] for t in ex.ticks]
    assert arr == sorted(arr)
    assert len(res) == len(trace)


def test_trace_rate_and_offsets():
    tr = serve.make_trace(64, 10.0, 25.0, seed=505)
    assert abs(len(tr) / (64 * 10.0) - 25.0) < 1.5
    firsts = {}
    for t, s, k in tr:
        firsts.setdefault(s, t)
    assert all(0 <= t < 0.04 for t in firsts.values())
    assert [t for t, _, _ in tr] == sorted(t for t, _, _ in tr)


def test_latency_stats():
    rs = [serve.Result(0, k, 0.0, k * 1e-3, None, None) for k in range(101)]
    st = serve.latency_stats(rs)
    assert st["frames"] == 101 and abs(st["p50_ms"] - 50) < 1e-9 and abs(st["p99_ms"] - 99) < 1e-9


class FakePipelinedExecutor:
    """Ticks in flight on a fake device: a tick submitted at time t starts
    when the previous tick's first stage has finished (stages of consecutive
    ticks overlap) and completes `tick_s` after its start; at most `depth`
    ticks are in flight.  Records the submit time of every tick and the
    number of ticks in flight at each submit."""

    def __init__(self, clock, tick_s=0.004, depth=2):
        self.clock, self.tick_s, self.depth = clock, tick_s, depth
        self.inflight = []          # (t_complete, frames)
        self.ticks, self.submits, self.live = [], [], set()
        self.ready = []

    def admit(self, spec):
        self.live.add(spec.sid)

    def evict(self, sid):
        self.ready += self.drain(lambda: self.clock.t)
        self.live.discard(sid)

    def busy(self):
        return bool(self.inflight)

    def can_submit(self):
        return len(self.inflight) < self.depth

    def submit(self, frames, now=None):
        assert self.can_submit() and all(f.sid in self.live for f in frames)
        t = self.clock.t
        start = max(t, self.inflight[-1][2] if self.inflight else t)
        self.submits.append((t, len(self.inflight)))
        self.ticks.append([(f.sid, f.k) for f in frames])
        # the next tick may start once this one's first half has run
        self.inflight.append((start + self.tick_s, frames, start + self.tick_s / 2))
        self.clock.t += 1e-5

    def _results(self, frames, t):
        return [serve.Result(f.sid, f.k, f.t_arrival, t, np.zeros((0, 4), np.float32),
                             np.zeros(0, np.int32)) for f in frames]

    def poll(self, now):
        out, self.ready = self.ready, []
        while self.inflight and self.inflight[0][0] <= self.clock.t:
            _, frames, _ = self.inflight.pop(0)
            out += self._results(frames, now())
        return out

    def wait_until(self, stop, now=None):
        if self.inflight and not stop():
            self.clock.t = max(self.clock.t, self.inflight[0][0])

    def drain(self, now):
        out = []
        while self.inflight:
            tc, frames, _ = self.inflight.pop(0)
            self.clock.t = max(self.clock.t, tc)
            out += self._results(frames, now())
        return out


def test_pipelined_loop_overlaps_ticks_and_keeps_order():
    """Frames that arrive while a tick is in flight are submitted before it
    completes (two ticks in flight), never more than `depth`; every frame
    gets a result, each stream's frames in order, none before its tick is
    done."""
    clock = FakeClock()
    ex = FakePipelinedExecutor(clock, tick_s=0.02, depth=2)
    sch = serve.Scheduler(budget=10**9, max_jobs=64, max_points=10**6, footprint=fp_const(10))
    trace = serve.make_trace(6, 1.0, 25.0, seed=3, rate_scale=3.0)
    res = serve.run_trace(trace, frame_fn, [spec(s) for s in range(6)], sch, ex, clock=clock,
                          sleep=clock.sleep)
    assert len(res) == len(trace)
    assert sorted((r.sid, r.k) for r in res) == sorted((s, k) for _, s, k in trace)
    assert max(n for _, n in ex.submits) == 1          # submitted with one tick in flight
    assert sum(1 for _, n in ex.submits if n == 1) > 0.2 * len(ex.submits)
    last = {}
    for tick in ex.ticks:
        assert len({s for s, _ in tick}) == len(tick)
        for s, k in tick:
            assert k == last.get(s, -1) + 1
            last[s] = k
    assert all(r.latency >= 0.02 - 1e-9 for r in res)


def test_pipelined_loop_depth_one_is_blocking():
    clock = FakeClock()
    ex = FakePipelinedExecutor(clock, tick_s=0.02, depth=1)
    sch = serve.Scheduler(budget=10**9, max_jobs=64, max_points=10**6, footprint=fp_const(10))
    trace = serve.make_trace(4, 0.5, 25.0, seed=4, rate_scale=2.0)
    res = serve.run_trace(trace, frame_fn, [spec(s) for s in range(4)], sch, ex, clock=clock,
                          sleep=clock.sleep)
    assert len(res) == len(trace)
    assert all(n == 0 for _, n in ex.submits)


def test_check_frame_refuses_what_the_upload_would_overrun():
    import torch

    spec = serve.StreamSpec(sid=3, W=6, H=4, levels=2, n_max=5, m_max=2)
    good = [torch.zeros((4, 6), dtype=torch.uint8), np.zeros((4, 6), np.uint8)]
    seeds = (np.zeros((5, 2), np.float32), np.zeros(5, np.int32), np.zeros((2, 4), np.float32))
    for px in good:
        serve.check_frame(serve.Frame(3, 0, 0.0, px), spec)
        serve.check_frame(serve.Frame(3, 0, 0.0, px, seeds), spec)
    for px in (torch.zeros((4, 7), dtype=torch.uint8), torch.zeros((4, 6), dtype=torch.int16),
               torch.zeros((6, 4), dtype=torch.uint8).t(), np.zeros((5, 6), np.uint8),
               np.zeros((4, 6), np.float32), None):
        with pytest.raises(ValueError, match="pixels"):
            serve.check_frame(serve.Frame(3, 1, 0.0, px), spec)
    bad_seeds = [
        (np.zeros((5, 3), np.float32), np.zeros(5, np.int32), np.zeros((2, 4), np.float32)),
        (np.zeros((5, 2), np.float32), np.zeros(4, np.int32), np.zeros((2, 4), np.float32)),
        (np.zeros((5, 2), np.float32), np.zeros(5, np.int32), np.zeros((2, 5), np.float32)),
        (np.zeros((6, 2), np.float32), np.zeros(6, np.int32), np.zeros((2, 4), np.float32)),
        (np.zeros((5, 2), np.float32), np.zeros(5, np.int32), np.zeros((3, 4), np.float32)),
    ]
    for sd in bad_seeds:
        with pytest.raises(ValueError, match="detections"):
            serve.check_frame(serve.Frame(3, 2, 0.0, good[0], sd), spec)
