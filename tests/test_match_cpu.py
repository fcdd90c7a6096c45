"""Host side of the matching and update phases (the library's optimal
assignment and track update, no GPU needed) against the oracle, plus the
argument checks of the IoU entry point (nothing is launched)."""
import os

import numpy as np
import pytest

import oracle
from paper_1910_06017_amd import ops

FAKE = 0x7F0000000000


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ops.LIB_PATH):
        pytest.skip("libomnitrack.so not built")
    return ops.lib()


def err(name):
    return {v: k for k, v in ops.ERRORS.items()}[name]


def valid(w, thr, s2d, d2s, score):
    tot = 0.0
    for i, j in enumerate(s2d):
        if j >= 0:
            assert d2s[j] == i and w[i, j] >= thr
            tot += float(w[i, j])
    for j, i in enumerate(d2s):
        if i >= 0:
            assert s2d[i] == j
    assert abs(tot - score) < 1e-9


@pytest.mark.parametrize("seed", range(4))
def test_assign_matches_oracle(L, seed):
    """Same float32 matrix, same float32 threshold decision on both sides:
    the optimal sums agree; random continuous scores have a unique optimum,
    so the matchings agree too."""
    rng = np.random.default_rng(seed)
    for _ in range(150):
        m, k = (int(v) for v in rng.integers(0, 12, 2))
        w = (rng.uniform(0, 1, (m, k)) * (rng.uniform(size=(m, k)) < 0.5)).astype(np.float32)
        thr = float(rng.choice([0.1, 0.3, 0.5]))
        s2d, d2s, score = ops.assign(w, thr)
        o = oracle.assign(w.astype(np.float64), float(np.float32(thr)))
        valid(w, np.float32(thr), s2d, d2s, score)
        assert abs(score - o[2]) < 1e-9
        assert np.array_equal(s2d, o[0]) and np.array_equal(d2s, o[1])


def test_assign_large_and_rectangular(L):
    rng = np.random.default_rng(9)
    for m, k in [(64, 64), (200, 37), (37, 200), (300, 300)]:
        w = rng.uniform(0, 1, (m, k)).astype(np.float32)
        w[rng.uniform(size=(m, k)) < 0.7] = 0
        s2d, d2s, score = ops.assign(w, 0.3)
        o = oracle.assign(w.astype(np.float64), float(np.float32(0.3)))
        valid(w, np.float32(0.3), s2d, d2s, score)
        assert abs(score - o[2]) < 1e-9


def test_assign_ties_and_edges(L):
    # duplicate detections: two optimal matchings, either is fine
    w = np.array([[0.8, 0.8], [0.0, 0.0]], np.float32)
    s2d, d2s, score = ops.assign(w, 0.3)
    assert abs(score - 0.8) < 1e-7 and s2d[1] == -1 and s2d[0] in (0, 1)
    # the greedy counterexample
    w = np.array([[0.9, 0.8], [0.85, 0.0]], np.float32)
    s2d, d2s, score = ops.assign(w, 0.3)
    assert s2d.tolist() == [1, 0] and d2s.tolist() == [1, 0]
    # inclusive threshold, everything below it unmatched
    w = np.array([[0.5, 0.49]], np.float32)
    assert ops.assign(w, 0.5)[0].tolist() == [0]
    assert ops.assign(w, 0.51)[0].tolist() == [-1]
    assert ops.assign(np.zeros((3, 0), np.float32), 0.3)[0].tolist() == [-1, -1, -1]
    assert ops.assign(np.zeros((0, 4), np.float32), 0.3)[1].tolist() == [-1] * 4
    E = err("OT_E_INVAL")
    s = np.zeros(2, np.int32)
    for thr in (0.0, -0.1, 1.5, float("nan")):
        assert L.ot_assign(w.ctypes.data, 1, 2, thr, s.ctypes.data, s.ctypes.data, None) == E
    assert L.ot_assign(None, 1, 2, 0.3, s.ctypes.data, s.ctypes.data, None) == E
    assert L.ot_assign(w.ctypes.data, -1, 2, 0.3, s.ctypes.data, s.ctypes.data, None) == E


def scenario(seed, m, k, cap_extra=8):
    rng = np.random.default_rng(seed)
    boxes = rng.uniform(0, 500, (m, 4)).astype(np.float32)
    ids = rng.permutation(1000)[:m].astype(np.int32)
    lost = (rng.uniform(size=m) < 0.2).astype(np.uint8)
    det = rng.uniform(0, 500, (k, 4)).astype(np.float32)
    w = rng.uniform(0, 1, (m, k)).astype(np.float32)
    w[lost == 1] = 0
    s2d, d2s, _ = ops.assign(w, 0.4)
    return boxes, ids, lost, det, s2d, d2s


@pytest.mark.parametrize("seed,m,k", [(1, 10, 12), (2, 12, 5), (3, 0, 4), (4, 6, 0), (5, 30, 30)])
def test_track_update_matches_oracle(L, seed, m, k):
    boxes, ids, lost, det, s2d, d2s = scenario(seed, m, k)
    cap = m + k
    B = np.zeros((cap, 4), np.float32)
    I = np.zeros(cap, np.int32)
    S = np.zeros(cap, np.uint8)
    B[:m], I[:m], S[:m] = boxes, ids, lost
    mo, nid = ops.track_update(B, I, S, m, det, s2d, d2s, 5000)
    ob, oi, ol, onid = oracle.track_update(boxes, ids, lost, det, s2d, d2s, 5000)
    assert mo == len(ob) and nid == onid
    assert np.array_equal(B[:mo], ob.astype(np.float32))
    assert np.array_equal(I[:mo], oi) and np.array_equal(S[:mo], ol)


def test_track_update_errors(L):
    boxes, ids, lost, det, s2d, d2s = scenario(7, 8, 9)
    fresh = int((d2s < 0).sum())
    cap = 8 + fresh - 1                      # one slot short
    B = np.zeros((cap, 4), np.float32)
    I = np.zeros(cap, np.int32)
    S = np.zeros(cap, np.uint8)
    B[:8], I[:8], S[:8] = boxes, ids, lost
    before = (B.copy(), I.copy(), S.copy())
    with pytest.raises(ops.OtError) as e:
        ops.track_update(B, I, S, 8, det, s2d, d2s, 0)
    assert e.value.code == err("OT_E_WORKSPACE")
    assert all(np.array_equal(a, b) for a, b in zip((B, I, S), before))
    bad = s2d.copy()
    j = int(np.where(bad >= 0)[0][0])
    bad[j] = (bad[j] + 1) % 9                # no longer mutual with d2s
    B2 = np.zeros((40, 4), np.float32)
    with pytest.raises(ops.OtError) as e:
        ops.track_update(B2, np.zeros(40, np.int32), np.zeros(40, np.uint8), 8, det, bad, d2s, 0)
    assert e.value.code == err("OT_E_INVAL")


def test_iou_matrix_validation(L):
    E = err("OT_E_INVAL")
    assert L.ot_iou_matrix(FAKE, -1, FAKE, 3, None, FAKE, None) == E
    assert L.ot_iou_matrix(FAKE + 4, 2, FAKE, 3, None, FAKE, None) == E     # S not 16-aligned
    assert L.ot_iou_matrix(FAKE, 2, FAKE + 8, 3, None, FAKE, None) == E     # D not 16-aligned
    assert L.ot_iou_matrix(FAKE, 2, FAKE, 3, None, None, None) == E
    assert L.ot_iou_matrix(None, 0, None, 3, None, None, None) == 0           # empty: no-op
