"""Materialized Scharr planes (OT_PYR_GRADS): the planes equal the oracle's
integer Scharr sums of every level, and tracking from a pyramid that carries
them gives bit-for-bit the results of the fused (per-point) gradients."""
import numpy as np
import pytest

import oracle
from paper_1910_06017_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06017_amd import ops as o
    o.lib()
    return o


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("shape,levels", [((1, 1), 3), ((5, 7), 4), ((33, 65), 5),
                                          ((576, 720), 4), ((17, 300), 8), ((1080, 1920), 5)])
def test_gradient_planes_match_oracle(ops, shape, levels):
    rng = np.random.default_rng(sum(shape) + 1)
    img = rng.integers(0, 256, shape).astype(np.uint8)
    P = ops.pyramid_build(dev(img), levels, grads=True)
    torch.cuda.synchronize()
    want = oracle.pyramid(img, levels)
    for l in range(levels):
        sx, sy = P.grads(l)
        wx, wy = oracle.scharr(want[l])
        assert np.array_equal(sx.cpu().numpy(), wx), f"level {l} sx"
        assert np.array_equal(sy.cpu().numpy(), wy), f"level {l} sy"
        if l > 0:
            assert np.array_equal(P.level(l).cpu().numpy(), want[l])


def track_both(ops, f0, f1, pts, win, levels, margin=0):
    P = ops.pyramid_build(dev(f0), levels)
    PG = ops.pyramid_build(dev(f0), levels, grads=True)
    Q = ops.pyramid_build(dev(f1), levels)
    p = dev(pts)
    a = ops.lk_track(P, Q, p, win=win, levels=levels, margin=margin, want_diag=True)
    b = ops.lk_track(PG, Q, p, win=win, levels=levels, margin=margin, want_diag=True)
    torch.cuda.synchronize()
    return a, b


@pytest.mark.parametrize("margin", [0, 4, 6, 2])
def test_tracking_with_planes_is_identical(ops, margin):
    w = synth.sd_boxes_workload()
    a, b = track_both(ops, w.frame0, w.frame1, w.pts, 21, w.levels, margin)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("win", [7, 15, 31])
def test_tracking_with_planes_other_windows(ops, win):
    w = synth.sd_shift_workload(seed=9)
    a, b = track_both(ops, w.frame0, w.frame1, w.pts, win, 3)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_tracking_with_planes_small_images_and_edges(ops):
    rng = np.random.default_rng(17)
    for (H, W) in [(24, 24), (40, 70), (9, 130)]:
        f0 = (rng.random((H, W)) * 255).astype(np.uint8)
        f1 = np.roll(f0, (1, -2), (0, 1))
        ys, xs = np.meshgrid(np.linspace(0, H - 1, 7), np.linspace(0, W - 1, 9), indexing="ij")
        pts = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.float32)
        a, b = track_both(ops, f0, f1, pts, 21, 3)
        for x, y in zip(a, b):
            assert torch.equal(x, y), (H, W)


def test_batched_accepts_prev_with_planes(ops):
    from paper_1910_06017_amd import batch
    ws = synth.batched_streams(seed=12, nstreams=3, npts_range=(100, 800), nbox_range=(1, 4))
    jobs = batch.jobs_from_workloads(ws)
    ref = []
    for j, w in zip(jobs, ws):
        Q = ops.pyramid_build(j.next_frame, w.levels)
        ref.append(ops.lk_track(j.prev, Q, j.pts, win=21, levels=w.levels))
        j.prev = ops.pyramid_build(dev(w.frame0), w.levels, grads=True)
    cfg = batch.BatchConfig(max_jobs=8, max_points=10000, max_boxes=64, max_tiles=4096)
    r = batch.BatchRunner(cfg)
    r.pack(jobs)
    r.run()
    torch.cuda.synchronize()
    for j, (nx, st, er) in zip(jobs, ref):
        assert torch.equal(j.next_pts, nx) and torch.equal(j.status, st)
