"""Tracking at a working level (the resolution-dependent pyramid level of
the preprocessing phase) on the GPU against the oracle: the same parity
classes and tolerances as full-resolution tracking (see test_gpu_parity)."""
import numpy as np
import pytest

import oracle
from paper_1910_06017_amd import synth
from test_gpu_parity import compare, dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06017_amd import ops as o
    o.lib()
    return o


def test_working_level_policy_matches_oracle(ops):
    for W in list(range(1, 3000, 37)) + [720, 1280, 1281, 1920, 2560, 2561, 3840, 7680]:
        for mw in (1280, 640, 333):
            assert ops.working_level(W, 100, mw) == oracle.working_level(W, 100, mw), (W, mw)


@pytest.mark.parametrize("eps", [0.01, 0.0])
def test_parity_hd_boxes_at_working_level(ops, eps):
    """1920x1080 goes to working level 1: levels 1..4 of a 5-level pyramid."""
    w = synth.hd_boxes_workload()
    base = ops.working_level(w.W, w.H)
    assert base == 1
    L = 4
    pts = w.pts[::3].copy()
    P = ops.pyramid_build(dev(w.frame0), base + L)
    Q = ops.pyramid_build(dev(w.frame1), base + L)
    g = ops.lk_track(P, Q, dev(pts), win=21, levels=L, iters=30, eps=eps, want_diag=True,
                     base_level=base)
    torch.cuda.synchronize()
    g = [t.cpu().numpy() for t in g]
    o = oracle.lk_track_working(w.frame0, w.frame1, pts, base, 21, L, 30,
                                float(np.float32(eps)))
    conv = None
    if eps == 0.0:
        o1 = oracle.lk_track_working(w.frame0, w.frame1, pts, base, 21, L, 30,
                                     float(np.float32(0.01)))
        conv = ~(o1.iters >= 30).any(1)
    compare(g, o, f"hd_boxes base {base} eps {eps}", eps=eps, o_conv=conv)


def test_working_level_zero_is_plain_tracking(ops):
    w = synth.sd_boxes_workload()
    P = ops.pyramid_build(dev(w.frame0), 4)
    Q = ops.pyramid_build(dev(w.frame1), 4)
    a = ops.lk_track(P, Q, dev(w.pts), levels=4)
    b = ops.lk_track(P, Q, dev(w.pts), levels=4, base_level=0)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_working_level_limits(ops):
    w = synth.sd_boxes_workload()
    P = ops.pyramid_build(dev(w.frame0), 4)
    Q = ops.pyramid_build(dev(w.frame1), 4)
    with pytest.raises(ops.OtError):
        ops.lk_track(P, Q, dev(w.pts), levels=3, base_level=2)   # needs 5 levels
    with pytest.raises(ops.OtError):
        ops.lk_track(P, Q, dev(w.pts), levels=1, base_level=-1)
    r = ops.lk_track(P, Q, dev(w.pts), levels=1, base_level=3)   # the coarsest level alone
    torch.cuda.synchronize()
    o = oracle.lk_track_working(w.frame0, w.frame1, w.pts, 3, 21, 1, 30, float(np.float32(0.01)))
    st = r[1].cpu().numpy()
    assert (st == o.status).mean() >= 0.999
