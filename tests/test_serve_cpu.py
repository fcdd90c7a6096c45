"""Serving scheduler on the CPU: admission by HBM budget, continuous batching,
eviction of silent streams, capacities, plain FIFO mode -- with a fake clock
and a fake executor (no GPU, no kernels)."""
import numpy as np

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
