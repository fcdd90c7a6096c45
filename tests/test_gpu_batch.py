"""Batched tick (one launch per stage over many streams) against the
per-stream calls and the oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1910_06017_amd import synth
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06017_amd import batch, ops
    ops.lib()
    return ops, batch


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_job(ops, batch, w, with_err=True):
    H, W = w.frame0.shape
    n, m = w.n, w.boxes.shape[0]
    prev = ops.pyramid_build(dev(w.frame0), w.levels)
    return batch.Job(prev=prev, next_frame=dev(w.frame1),
                     next_ws=ops.alloc_workspace(W, H, w.levels), levels=w.levels,
                     pts=dev(w.pts), next_pts=torch.full((n, 2), -7.0, device="cuda"),
                     status=torch.full((n,), 9, dtype=torch.uint8, device="cuda"),
                     err=torch.full((n,), -9.0, device="cuda") if with_err else None,
                     boxes=dev(w.boxes), box_id=dev(w.box_id),
                     out_boxes=torch.full((m, 4), -7.0, device="cuda"),
                     out_count=torch.full((m,), -1, dtype=torch.int32, device="cuda"))


def reference(ops, j, cfg):
    Q = ops.pyramid_build(j.next_frame, j.levels)
    nx, st, er = ops.lk_track(j.prev, Q, j.pts, win=cfg.win, levels=j.levels, iters=cfg.iters,
                              eps=cfg.eps, min_eig=cfg.min_eig, margin=cfg.margin)
    ob, oc = ops.box_update(j.boxes, j.box_id, j.pts, nx, st)
    return Q, nx, st, er, ob, oc


def small_mix(seed=11, nstreams=7):
    ws = synth.batched_streams(seed=seed, nstreams=nstreams, npts_range=(60, 3000),
                               nbox_range=(1, 8))
    # ragged cases: a stream without points and boxes, one with one point
    w0 = ws[0]
    ws.append(synth.Workload("empty", w0.frame0, w0.frame1, w0.pts[:0], w0.truth[:0],
                             w0.box_id[:0], w0.boxes[:0], w0.boxes_next[:0], 21, w0.levels))
    ws.append(synth.Workload("one", w0.frame0, w0.frame1, w0.pts[:1], w0.truth[:1],
                             w0.box_id[:1], w0.boxes[:1], w0.boxes_next[:1], 21, w0.levels))
    return ws


@pytest.mark.parametrize("sched", [dict(lk_waves=0, chunk=1), dict(lk_waves=0, exact_grids=True),
                                   dict(lk_waves=600, chunk=1), dict(lk_waves=600, exact_grids=True),
                                   dict(lk_waves=2048, chunk=3), dict(margin=2, lk_waves=0),
                                   dict(margin=4, lk_wpg=2, lk_ppw=1),
                                   dict(margin=4, lk_wpg=4, lk_ppw=2, exact_grids=True),
                                   dict(margin=6, lk_wpg=1, lk_ppw=4),
                                   dict(margin=6, lk_wpg=4, lk_ppw=4)])
def test_batched_equals_per_stream(mods, sched):
    ops, batch = mods
    ws = small_mix()
    cfg = batch.BatchConfig(max_jobs=16, max_points=40000, max_boxes=256, max_tiles=4096,
                            max_levels=5, **sched)
    jobs = [make_job(ops, batch, w, with_err=(i % 3 != 1)) for i, w in enumerate(ws)]
    runner = batch.BatchRunner(cfg)
    nxt = runner.pack(jobs)
    runner.run()
    torch.cuda.synchronize()
    for j, Qb, w in zip(jobs, nxt, ws):
        Q, nx, st, er, ob, oc = reference(ops, j, cfg)
        torch.cuda.synchronize()
        for l in range(1, j.levels):
            assert torch.equal(Qb.level(l), Q.level(l)), (w.name, l)
        assert torch.equal(j.next_pts, nx), w.name
        assert torch.equal(j.status, st), w.name
        if j.err is not None:
            assert torch.equal(j.err, er), w.name
        assert torch.equal(j.out_boxes, ob), w.name
        assert torch.equal(j.out_count, oc), w.name


def test_graph_replay_with_new_tables(mods):
    """One captured tick replayed with re-packed tables (different streams and
    sizes, same capacities) matches eager ticks; host work between replays."""
    ops, batch = mods
    cfg = batch.BatchConfig(max_jobs=8, max_points=30000, max_boxes=128, max_tiles=4096,
                            max_levels=5)
    runner = batch.BatchRunner(cfg, tables=1)
    mixes = [small_mix(seed=s, nstreams=4) for s in (21, 22, 23)]
    all_jobs = [[make_job(ops, batch, w) for w in ws] for ws in mixes]
    runner.pack(all_jobs[0], table=0)
    g = runner.capture(0)
    for rep in range(2):
        for jobs in all_jobs:
            for j in jobs:
                j.next_pts.fill_(-7.0)
                j.out_count.fill_(-1)
            torch.cuda.synchronize()
            runner.pack(jobs, table=0)
            g.replay()
            torch.cuda.synchronize()
            _ = np.random.default_rng(rep).normal(size=1000).sum()  # host work between replays
            for j in jobs:
                Q, nx, st, er, ob, oc = reference(ops, j, cfg)
                torch.cuda.synchronize()
                assert torch.equal(j.next_pts, nx)
                assert torch.equal(j.status, st)
                assert torch.equal(j.out_boxes, ob) and torch.equal(j.out_count, oc)


def test_graph_with_fitted_capacities(mods):
    """A tick captured with capacities fitted to its jobs (no idle workgroups
    in any stage) gives the per-stream results bit for bit, on every replay;
    a tick that needs more than the fitted capacities is refused at packing."""
    ops, batch = mods
    jobs = [make_job(ops, batch, w) for w in small_mix(seed=31, nstreams=5)]
    cfg = batch.fit_capacities(batch.BatchConfig(max_jobs=16, max_points=1 << 16,
                                                 max_boxes=512, max_tiles=1 << 14,
                                                 max_levels=5), jobs)
    assert cfg.max_points == sum(j.n for j in jobs) and cfg.max_boxes == sum(j.m for j in jobs)
    runner = batch.BatchRunner(cfg, tables=1)
    runner.pack(jobs, table=0)
    g = runner.capture(0)
    refs = [reference(ops, j, cfg) for j in jobs]
    for rep in range(3):
        for j in jobs:
            j.next_pts.fill_(-7.0)
            j.out_count.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for j, (Q, nx, st, er, ob, oc) in zip(jobs, refs):
            assert torch.equal(j.next_pts, nx), rep
            assert torch.equal(j.status, st)
            assert torch.equal(j.out_boxes, ob) and torch.equal(j.out_count, oc)
    bigger = jobs + [make_job(ops, batch, synth.batched_streams(seed=32, nstreams=1)[0])]
    with pytest.raises(ops.OtError):
        runner.pack(bigger, table=0)


def test_batched_full_tick_vs_oracle(mods):
    """The 32-stream mixed tick (~170k points) in the persistent launch against
    the oracle: every point of four streams (the largest stream, a 1080p, a
    720p and an SD stream) and a sample of 150 points of each other stream,
    all held to the single-call parity bar (every point within 0.01 px)."""
    ops, batch = mods
    ws = synth.batched_streams()
    cfg = batch.BatchConfig(max_jobs=32, max_points=1 << 18, max_boxes=1024, max_tiles=1 << 15,
                            max_levels=5, lk_waves=8192, chunk=2)
    jobs = [make_job(ops, batch, w) for w in ws]
    runner = batch.BatchRunner(cfg)
    runner.pack(jobs)
    runner.run()
    torch.cuda.synchronize()
    full = {int(np.argmax([w.n for w in ws]))}
    for W in (1920, 1280, 720):
        full.add(next(i for i, w in enumerate(ws) if w.frame0.shape[1] == W and i not in full))
    rng = np.random.default_rng(4)
    sel_all, g_all, o_all = [], [], []
    for s_i, (j, w, Qb) in enumerate(zip(jobs, ws, runner.next_pyrs)):
        sel = (np.arange(w.n) if s_i in full
               else np.sort(rng.choice(w.n, size=min(w.n, 150), replace=False)))
        o = oracle.lk_track(w.frame0, w.frame1, w.pts[sel], win=21, levels=w.levels, iters=30,
                            eps=float(np.float32(0.01)))
        # per-level iteration counts of the same points (single-call path, same bits)
        nx, st, er, it, _ = ops.lk_track(j.prev, Qb, dev(w.pts[sel]), win=21, levels=w.levels,
                                         want_diag=True)
        assert torch.equal(nx.cpu(), j.next_pts.cpu()[sel])
        assert torch.equal(st.cpu(), j.status.cpu()[sel])
        g = (j.next_pts.cpu().numpy()[sel], j.status.cpu().numpy()[sel],
             j.err.cpu().numpy()[sel], it.cpu().numpy(), None)
        tag = (f"batched stream {s_i} ({w.frame0.shape[1]}x{w.frame0.shape[0]}, "
               f"{'all' if s_i in full else 'sample of'} {len(sel)} points)")
        if s_i in full:
            compare(g, o, tag)
        else:
            sel_all.append(len(sel))
            g_all.append(g)
            o_all.append(o)
    # the sampled points of the other streams, pooled per level count
    for L in sorted({g[3].shape[1] for g in g_all}):
        idx = [i for i, g in enumerate(g_all) if g[3].shape[1] == L]
        gp = tuple(np.concatenate([g_all[i][k] for i in idx]) for k in range(4)) + (None,)
        op = type("O", (), {})()
        for k in ("next_pts", "status", "err", "iters"):
            setattr(op, k, np.concatenate([getattr(o_all[i], k) for i in idx]))
        compare(gp, op, f"batched, {sum(sel_all[i] for i in idx)} sampled points of "
                        f"{len(idx)} streams with {L} levels")


def test_batched_repeatable(mods):
    ops, batch = mods
    ws = small_mix(seed=31, nstreams=5)
    cfg = batch.BatchConfig(max_jobs=16, max_points=30000, max_boxes=256, lk_waves=1024,
                            chunk=2)
    jobs = [make_job(ops, batch, w) for w in ws]
    runner = batch.BatchRunner(cfg)
    outs = []
    for _ in range(4):
        runner.pack(jobs)
        runner.run()
        torch.cuda.synchronize()
        outs.append([(j.next_pts.clone(), j.status.clone(), j.out_boxes.clone()) for j in jobs])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert all(torch.equal(x, y) for x, y in zip(a, b))


def test_autotuner_picks_and_caches(mods, tmp_path):
    ops, batch = mods
    ws = small_mix(seed=41, nstreams=4)
    jobs = [make_job(ops, batch, w) for w in ws]
    tuner = batch.Autotuner(path=str(tmp_path / "tune.json"),
                            candidates=[{"margin": 4, "lk_waves": 0, "chunk": 1},
                                        {"margin": 3, "lk_waves": 1024, "chunk": 2}])
    base = batch.BatchConfig(max_jobs=16, max_points=30000, max_boxes=256)
    rec = tuner.tune(jobs, base, reps=3, warmup=1)
    assert rec["schedule"] in tuner.candidates
    again = batch.Autotuner(path=str(tmp_path / "tune.json"))
    assert again.best(batch.bucket_key(jobs)) == rec["schedule"]


def test_unsupported_shapes_are_rejected(mods):
    """Several waves or points per workgroup exist for the 21 x 21 window at
    margins 4 and 6 only, and not with the persistent grid."""
    ops, batch = mods
    ws = small_mix(seed=12, nstreams=2)
    jobs = [make_job(ops, batch, w) for w in ws]
    for sched in (dict(margin=3, lk_wpg=2), dict(margin=4, lk_wpg=3),
                  dict(margin=4, lk_ppw=2, lk_waves=512)):
        runner = batch.BatchRunner(batch.BatchConfig(max_jobs=16, max_points=40000,
                                                     max_boxes=256, **sched))
        runner.pack(jobs)
        with pytest.raises(ops.OtError) as e:
            runner.run()
        assert e.value.code == -5
