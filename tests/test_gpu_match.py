"""Matching phase on the GPU: the IoU score matrix against the oracle, and
the whole matching/update step (GPU scores, host assignment and update)
against the oracle on the same scores.

IoU in float32 takes a handful of roundings of values below 2^11 px, so it
lies within 1e-6 of the FP64 value.  The assignment's threshold decision
is taken on the float32 scores on both sides (the oracle gets the float32
matrix and the float32 threshold), so the optimal sums agree to rounding
of the summation; random scores have a unique optimum, so the matchings and
the updated object lists agree exactly."""
import numpy as np
import pytest

import oracle
from paper_1910_06017_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

IOU_ATOL = 1e-6


@pytest.fixture(scope="module")
def ops():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06017_amd import ops as o
    o.lib()
    return o


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def boxes_with_overlaps(seed, m, k):
    """Detections mostly near the objects (so scores span 0..1), a few far
    away, some degenerate and inverted boxes."""
    rng = np.random.default_rng(seed)
    xy = rng.uniform([0, 0], [1900, 1060], (m, 2))
    S = np.concatenate([xy, xy + rng.uniform(1, 300, (m, 2))], axis=1)
    near = rng.integers(0, max(m, 1), k) if m else np.zeros(k, int)
    D = (S[near] if m else np.zeros((k, 4))) + rng.normal(0, 20, (k, 4))
    far = rng.uniform(size=k) < 0.2
    D[far] = rng.uniform(0, 1900, (int(far.sum()), 4))
    if m:
        S[0, 2] = S[0, 0]                  # zero width
    if k > 1:
        D[1, [0, 2]] = D[1, [2, 0]]        # inverted
    return S.astype(np.float32), D.astype(np.float32)


@pytest.mark.parametrize("m,k,seed", [(1, 1, 1), (7, 13, 2), (30, 30, 3), (257, 129, 4),
                                      (1000, 37, 5)])
def test_iou_matrix_matches_oracle(ops, m, k, seed):
    S, D = boxes_with_overlaps(seed, m, k)
    rng = np.random.default_rng(seed + 100)
    act = (rng.uniform(size=m) >= 0.1).astype(np.uint8)
    g = ops.iou_matrix(dev(S), dev(D)).cpu().numpy()
    ga = ops.iou_matrix(dev(S), dev(D), active=dev(act)).cpu().numpy()
    o = oracle.iou_matrix(S, D)
    np.testing.assert_allclose(g, o, atol=IOU_ATOL, rtol=0)
    assert np.all(ga[act == 0] == 0) and np.array_equal(ga[act == 1], g[act == 1])
    assert np.all((g >= 0) & (g <= 1))
    assert (o > 0.3).sum() > 0 or m * k < 4


def test_iou_exact_cases(ops):
    S = np.array([[0, 0, 4, 4], [0, 0, 2, 1], [0, 0, 4, 4], [0, 1, 4, 2]], np.float32)
    D = np.array([[0, 0, 4, 4], [1, 0, 3, 1], [1, 1, 3, 3], [1, 0, 2, 4]], np.float32)
    g = ops.iou_matrix(dev(S), dev(D)).cpu().numpy()
    assert g[0, 0] == 1.0 and g[2, 2] == 0.25
    assert abs(g[1, 1] - 1 / 3) < 1e-7 and abs(g[3, 3] - 1 / 7) < 1e-7
    e = torch.zeros((0, 4), dtype=torch.float32, device="cuda")
    assert ops.iou_matrix(e, dev(D)).shape == (0, 4)


def test_match_update_step_sd_boxes(ops):
    """Predicted boxes from the tracking path on the 720x576 box scene,
    detections = true next boxes (1 px jitter, 10 % missed, 2 new): scores
    on the GPU, assignment and update through the library's host calls."""
    w = synth.sd_boxes_workload()
    P = ops.pyramid_build(dev(w.frame0), w.levels)
    Q = ops.pyramid_build(dev(w.frame1), w.levels)
    pts = dev(w.pts)
    nxt, st, _ = ops.lk_track(P, Q, pts, win=w.win, levels=w.levels, iters=w.iters, eps=w.eps)
    pred, _ = ops.box_update(dev(w.boxes), dev(w.box_id), pts, nxt, st)
    m = pred.shape[0]
    rng = np.random.default_rng(77)
    det = synth.detections(w.boxes_next, rng, w.W, w.H)
    lost0 = np.zeros(m, np.uint8)
    lost0[[3, 11]] = 1                                 # two objects lost earlier
    iou = ops.iou_matrix(pred, dev(det), active=dev(1 - lost0)).cpu().numpy()
    pred_h = pred.cpu().numpy()
    o_iou = oracle.iou_matrix(pred_h, det, active=1 - lost0)
    np.testing.assert_allclose(iou, o_iou, atol=IOU_ATOL)
    thr = 0.3
    s2d, d2s, score = ops.assign(iou, thr)
    o = oracle.assign(iou.astype(np.float64), float(np.float32(thr)))
    assert abs(score - o[2]) < 1e-9
    assert np.array_equal(s2d, o[0]) and np.array_equal(d2s, o[1])
    cap = m + det.shape[0]
    B = np.zeros((cap, 4), np.float32)
    I = np.zeros(cap, np.int32)
    L = np.zeros(cap, np.uint8)
    B[:m], I[:m], L[:m] = pred_h, np.arange(m), lost0
    mo, nid = ops.track_update(B, I, L, m, det, s2d, d2s, m)
    ob, oi, ol, onid = oracle.track_update(pred_h, np.arange(m), lost0, det, s2d, d2s, m)
    assert mo == len(ob) and nid == onid
    assert np.array_equal(B[:mo], ob.astype(np.float32))
    assert np.array_equal(I[:mo], oi) and np.array_equal(L[:mo], ol)
    matched = int((s2d >= 0).sum())
    print(f"match sd_boxes: {m} objects ({int(lost0.sum())} lost before), {len(det)} detections, "
          f"{matched} matched, score {score:.3f}, {mo - m} new, {int(ol[:m].sum())} lost after")
    assert matched >= 0.7 * (m - lost0.sum()) - 2
