"""HIP path vs the CPU oracle, element by element, through the C ABI.

Pyramids must match bit for bit.  Lucas-Kanade (FP32 on the GPU, FP64 in the
oracle) must agree on status for >= 99.9 % of the points, and every point
both calls tracked must lie within 0.01 px of the oracle, whatever its
class: converged with the same stopping decisions, a decision flip (an eps
test on the other side of the threshold, so the runs stop one iteration
apart), or capped (a level ran all `iters` iterations without converging).
The classes are reported for every comparison (sizes and maxima, also in
the session's terminal summary).  err is compared on the converged class.
Box updates must match within 0.01 px.
"""
import math

import numpy as np
import pytest

import oracle
import parity_log
from paper_1910_06017_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FLOW_TOL = 0.01      # px, every point tracked by both
STATUS_AGREE = 0.999
ERR_TOL = 0.01       # gray levels, converged points


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06017_amd import ops as o
    o.lib()
    return o


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_gpu(ops, f0, f1, pts, win, levels, iters, eps, diag=True, margin=0):
    P = ops.pyramid_build(dev(f0), levels)
    Q = ops.pyramid_build(dev(f1), levels)
    out = ops.lk_track(P, Q, dev(pts), win=win, levels=levels, iters=iters, eps=eps,
                       want_diag=diag, margin=margin)
    torch.cuda.synchronize()
    return [None if t is None else t.cpu().numpy() for t in out]


def run_oracle(f0, f1, pts, win, levels, iters, eps):
    return oracle.lk_track(f0, f1, pts, win=win, levels=levels, iters=iters,
                           eps=float(np.float32(eps)))


def compare(g, o, tag, flow_tol=FLOW_TOL, agree=STATUS_AGREE, err_tol=ERR_TOL, eps=0.01,
            iters=30, max_flip_frac=0.01, o_conv=None):
    """g = (next_pts, status, err[, iters, lam]) from the GPU; o = oracle result.

    Every point tracked by both must lie within flow_tol.  The points fall in
    three reported classes: converged with the same stopping decisions
    (every level stopped by the eps test at the same iteration), decision
    flips (an eps test on the other side of the threshold; at most
    max_flip_frac of the points) and capped (a level ran all `iters`
    iterations).  With eps = 0 every level runs `iters`; `o_conv` (the
    oracle run with eps 0.01 did not hit the cap) then marks the converged
    points.  err must agree within err_tol on the converged class."""
    gn, gs, ge = g[0], g[1], g[2]
    n = len(gs)
    ag = (gs == o.status).mean() if n else 1.0
    both = (gs == 1) & (o.status == 1)
    d = np.hypot(*(gn.astype(np.float64) - o.next_pts).T)
    gi = g[3].astype(np.int64) if len(g) > 3 and g[3] is not None else o.iters
    if eps > 0:
        capped = (o.iters >= iters).any(1) | (gi >= iters).any(1)
        same = np.all(gi == o.iters, axis=1)
    else:
        capped = ~o_conv if o_conv is not None else np.zeros(n, bool)
        same = np.ones(n, bool)
    conv = both & ~capped & same
    flip = both & ~capped & ~same
    cap = both & capped
    mx = lambda m: d[m].max() if m.any() else 0.0
    de = np.abs(ge.astype(np.float64) - o.err)
    emx = lambda m: de[m].max() if m.any() else 0.0
    msg = (f"{tag}: n={n} status agree={ag:.5f} tracked={both.sum()} | converged={conv.sum()} "
           f"max={mx(conv):.2e} px | flips={flip.sum()} max={mx(flip):.2e} px | "
           f"capped={cap.sum()} max={mx(cap):.2e} px | all max={mx(both):.2e} px (bar "
           f"{flow_tol}) | err max converged={emx(conv):.2e} capped={emx(cap):.2e} gray")
    parity_log.record(msg)
    assert ag >= agree, msg
    assert mx(both) <= flow_tol, msg
    assert flip.sum() <= max_flip_frac * max(1, both.sum()), msg
    if err_tol is not None:
        assert emx(conv) <= err_tol, msg
    assert np.all(ge[gs == 0] == -1.0)
    return d


# ------------------------------------------------------------------ pyramid
@pytest.mark.parametrize("shape,levels", [((1, 1), 3), ((5, 7), 4), ((33, 65), 5),
                                          ((576, 720), 5), ((1080, 1920), 6), ((17, 300), 8)])
def test_pyramid_bitexact(ops, shape, levels):
    rng = np.random.default_rng(sum(shape))
    img = rng.integers(0, 256, shape).astype(np.uint8)
    P = ops.pyramid_build(dev(img), levels)
    torch.cuda.synchronize()
    want = oracle.pyramid(img, levels)
    for l in range(1, levels):
        assert np.array_equal(P.level(l).cpu().numpy(), want[l]), f"level {l}"


def test_pyramid_pitched_frame(ops):
    rng = np.random.default_rng(5)
    big = rng.integers(0, 256, (200, 333)).astype(np.uint8)
    t = dev(big)[:, 7:7 + 250]           # row pitch 333 > width 250
    assert t.stride(0) == 333
    import ctypes as C
    ws = ops.alloc_workspace(250, 200, 4)
    d = ops.OtPyr()
    ops.check(ops.lib().ot_pyramid_build(t.data_ptr(), 250, 200, 333, 4, ws.data_ptr(),
                                         ws.numel(), 0, C.byref(d),
                                         torch.cuda.current_stream().cuda_stream), "build")
    torch.cuda.synchronize()
    P = ops.Pyramid(t, ws, d)
    want = oracle.pyramid(np.ascontiguousarray(big[:, 7:257]), 4)
    for l in range(1, 4):
        assert np.array_equal(P.level(l).cpu().numpy(), want[l])


# ------------------------------------------------------------------ Lucas-Kanade
def test_zero_motion_exact(ops):
    w = synth.sd_shift_workload(seed=3)
    g = run_gpu(ops, w.frame0, w.frame0, w.pts, 21, 3, 30, 0.01)
    ok = g[1] == 1
    assert ok.mean() > 0.95
    assert np.array_equal(g[0][ok], w.pts[ok])
    assert np.all(g[2][ok] == 0.0)


def conv_mask(w, win=21):
    o = run_oracle(w.frame0, w.frame1, w.pts, win, w.levels, w.iters, 0.01)
    return ~(o.iters >= w.iters).any(1)


@pytest.mark.parametrize("eps", [0.01, 0.0])
def test_parity_sd_shift(ops, eps):
    w = synth.sd_shift_workload()
    g = run_gpu(ops, w.frame0, w.frame1, w.pts, w.win, w.levels, w.iters, eps)
    o = run_oracle(w.frame0, w.frame1, w.pts, w.win, w.levels, w.iters, eps)
    compare(g, o, f"sd_shift eps={eps}", eps=eps, o_conv=conv_mask(w) if eps == 0 else None)


@pytest.mark.parametrize("eps", [0.01, 0.0])
def test_parity_sd_boxes(ops, eps):
    w = synth.sd_boxes_workload()
    g = run_gpu(ops, w.frame0, w.frame1, w.pts, w.win, w.levels, w.iters, eps)
    o = run_oracle(w.frame0, w.frame1, w.pts, w.win, w.levels, w.iters, eps)
    compare(g, o, f"sd_boxes eps={eps}", eps=eps, o_conv=conv_mask(w) if eps == 0 else None)


@pytest.mark.parametrize("eps", [0.01, 0.0])
def test_parity_hd_boxes(ops, eps):
    w = synth.hd_boxes_workload()
    g = run_gpu(ops, w.frame0, w.frame1, w.pts, w.win, w.levels, w.iters, eps)
    o = run_oracle(w.frame0, w.frame1, w.pts, w.win, w.levels, w.iters, eps)
    compare(g, o, f"hd_boxes eps={eps}", eps=eps, o_conv=conv_mask(w) if eps == 0 else None)


@pytest.mark.parametrize("win", [3, 5, 7, 9, 11, 13, 15, 17, 19, 23, 25, 29, 31])
def test_parity_window_sizes(ops, win):
    f0, f1, _ = synth.shifted_pair(40 + win, 160, 120, shift=(1.3, -0.7), mode="analytic")
    g = np.arange(2.5, 158, 9.0)
    pts = np.array([(x, y) for x in g for y in g if y < 119], np.float32)
    gg = run_gpu(ops, f0, f1, pts, win, 3, 20, 0.0)
    o = run_oracle(f0, f1, pts, win, 3, 20, 0.0)
    oc = run_oracle(f0, f1, pts, win, 3, 20, 0.01)
    compare(gg, o, f"win={win}", eps=0.0, iters=20, o_conv=~(oc.iters >= 20).any(1))


def test_parity_tiny_images_and_edges(ops):
    """Images smaller than the window, points on the border, ragged sizes."""
    rng = np.random.default_rng(9)
    for (H, W) in [(1, 1), (2, 3), (9, 13), (31, 17)]:
        a = rng.integers(0, 256, (H, W)).astype(np.uint8)
        b = np.roll(a, 1, axis=1)
        pts = np.array([[0, 0], [W - 1, H - 1], [(W - 1) / 2, (H - 1) / 2], [W - 1, 0]],
                       np.float32)
        g = run_gpu(ops, a, b, pts, 7, 2, 10, 0.0)
        o = run_oracle(a, b, pts, 7, 2, 10, 0.0)
        compare(g, o, f"tiny {H}x{W}", agree=1.0, flow_tol=1e-3, eps=0.0, iters=10)


def test_invalid_points(ops):
    w = synth.sd_shift_workload()
    pts = np.array([[-1, 5], [720, 5], [5, 576], [np.nan, 3], [3, np.inf], [100.5, 200.25]],
                   np.float32)
    g = run_gpu(ops, w.frame0, w.frame1, pts, 21, 3, 30, 0.01)
    assert list(g[1]) == [0, 0, 0, 0, 0, 1]
    assert np.all(g[3][:5] == 0)
    assert np.all(g[2][:5] == -1.0)


def test_iteration_counts_match(ops):
    w = synth.sd_shift_workload()
    gg = run_gpu(ops, w.frame0, w.frame1, w.pts, 21, 3, 30, 0.0, diag=True)
    o = run_oracle(w.frame0, w.frame1, w.pts, 21, 3, 30, 0.0)
    ok = (gg[1] == 1) & (o.status == 1)
    assert np.all(gg[3][ok] == 30)
    lam_g, lam_o = gg[4][ok], o.lam[ok]
    assert np.allclose(lam_g, lam_o, rtol=1e-4, atol=1e-3)


@pytest.mark.parametrize("margin", [1, 2, 8, 16])
def test_margin_does_not_change_results(ops, margin):
    w = synth.sd_boxes_workload()
    sel = slice(0, 2000)
    a = run_gpu(ops, w.frame0, w.frame1, w.pts[sel], 21, 4, 30, 0.01, diag=False)
    b = run_gpu(ops, w.frame0, w.frame1, w.pts[sel], 21, 4, 30, 0.01, margin=margin, diag=False)
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])


def test_order_does_not_change_results(ops):
    """Tracking the points in any processing order gives the same bits at
    the points' own indices; lk_order lists every point once, by descending
    total iterations."""
    w = synth.sd_boxes_workload()
    P = ops.pyramid_build(dev(w.frame0), 4)
    Q = ops.pyramid_build(dev(w.frame1), 4)
    pts = dev(w.pts)
    a = ops.lk_track(P, Q, pts, win=21, levels=4, want_diag=True)
    perm = dev(np.random.default_rng(8).permutation(w.n).astype(np.int32))
    b = ops.lk_track(P, Q, pts, win=21, levels=4, want_diag=True, order=perm)
    order = ops.lk_order(a[3])
    c = ops.lk_track(P, Q, pts, win=21, levels=4, want_diag=True, order=order)
    torch.cuda.synchronize()
    for x, y, z in zip(a, b, c):
        assert torch.equal(x, y) and torch.equal(x, z)
    o = order.cpu().numpy()
    assert np.array_equal(np.sort(o), np.arange(w.n))
    cost = a[3].cpu().numpy().astype(np.int64).sum(1)[o]
    assert np.all(np.diff(cost) <= 0)


def test_deterministic(ops):
    w = synth.sd_boxes_workload()
    a = run_gpu(ops, w.frame0, w.frame1, w.pts, 21, 4, 30, 0.01)
    for _ in range(3):
        b = run_gpu(ops, w.frame0, w.frame1, w.pts, 21, 4, 30, 0.01)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


# ------------------------------------------------------------------ box update
def test_box_update_parity_same_inputs(ops):
    rng = np.random.default_rng(12)
    # per-box tracked counts span the one-wave sort (<= 512), radix selection
    # on the gathered values (<= 6144) and radix selection re-scanning memory
    for trial, (m, n) in enumerate([(1, 0), (3, 1), (5, 200), (20, 8000), (4, 20000),
                                    (2, 30000)]):
        boxes = rng.uniform(0, 500, (m, 4)).astype(np.float32)
        box_id = rng.integers(-1, m, n).astype(np.int32)
        pts = rng.uniform(0, 700, (n, 2)).astype(np.float32)
        nxt = (pts + rng.normal(0, 4, (n, 2))).astype(np.float32)
        st = (rng.uniform(size=n) < 0.9).astype(np.uint8)
        ob, oc = ops.box_update(dev(boxes), dev(box_id), dev(pts), dev(nxt), dev(st))
        torch.cuda.synchronize()
        wb, wc = oracle.box_update(boxes, box_id, pts, nxt, st)
        assert np.array_equal(oc.cpu().numpy(), wc)
        assert np.allclose(ob.cpu().numpy(), wb, atol=1e-4, rtol=0), trial


def test_box_update_path_boundaries_and_ties(ops):
    """Boxes with exactly 511, 512, 513, 6144 and 6145 tracked points (the
    switch between the register sort, radix selection in LDS and radix
    selection from memory), with many equal displacements, zeros and signs."""
    rng = np.random.default_rng(13)
    counts = [511, 512, 513, 6144, 6145, 2]
    box_id = np.concatenate([np.full(c, b, np.int32) for b, c in enumerate(counts)])
    n, m = box_id.size, len(counts)
    rng.shuffle(box_id)
    pts = rng.uniform(0, 700, (n, 2)).astype(np.float32)
    d = rng.integers(-3, 4, (n, 2)).astype(np.float32) * 0.25   # few distinct values
    d[rng.uniform(size=n) < 0.1] = 0.0
    nxt = (pts + d).astype(np.float32)
    st = np.ones(n, np.uint8)
    boxes = rng.uniform(0, 500, (m, 4)).astype(np.float32)
    ob, oc = ops.box_update(dev(boxes), dev(box_id), dev(pts), dev(nxt), dev(st))
    torch.cuda.synchronize()
    wb, wc = oracle.box_update(boxes, box_id, pts, nxt, st)
    assert np.array_equal(oc.cpu().numpy(), wc)
    assert np.allclose(ob.cpu().numpy(), wb, atol=1e-4, rtol=0)


def test_box_update_end_to_end(ops):
    w = synth.sd_boxes_workload()
    P = ops.pyramid_build(dev(w.frame0), 4)
    Q = ops.pyramid_build(dev(w.frame1), 4)
    pts = dev(w.pts)
    nxt, st, err = ops.lk_track(P, Q, pts, win=21, levels=4)
    ob, oc = ops.box_update(dev(w.boxes), dev(w.box_id), pts, nxt, st)
    torch.cuda.synchronize()
    o = run_oracle(w.frame0, w.frame1, w.pts, 21, 4, 30, 0.01)
    wb, wc = oracle.box_update(w.boxes, w.box_id, w.pts, o.next_pts, o.status)
    same = oc.cpu().numpy() == wc
    # every box median is taken over points within 0.01 px of the oracle's
    d = np.abs(ob.cpu().numpy() - wb)[same]
    parity_log.record(f"sd_boxes box update end to end: counts equal {same.mean():.4f}, "
                      f"max corner difference {d.max():.2e} px")
    assert same.mean() >= 0.99
    assert d.max() <= FLOW_TOL, d.max()


# ------------------------------------------------------------------ ABI errors
def test_errors_leave_outputs_untouched(ops):
    w = synth.sd_shift_workload()
    P = ops.pyramid_build(dev(w.frame0), 3)
    Q = ops.pyramid_build(dev(w.frame1), 3)
    pts = dev(w.pts)
    n = len(w.pts)
    nxt = torch.full((n, 2), 7.0, device="cuda")
    st = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
    err = torch.full((n,), 5.0, device="cuda")
    for kw in [dict(win=20), dict(levels=4), dict(iters=0), dict(eps=-1.0)]:
        args = dict(win=21, levels=3, iters=30, eps=0.01)
        args.update(kw)
        with pytest.raises(ops.OtError):
            ops.lk_track(P, Q, pts, out=(nxt, st, err), **args)
    torch.cuda.synchronize()
    assert torch.all(nxt == 7.0) and torch.all(st == 9) and torch.all(err == 5.0)
    ops.lk_track(P, Q, pts[:0], out=(nxt[:0], st[:0], err[:0]))  # n == 0: no-op
