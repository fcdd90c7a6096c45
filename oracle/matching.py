"""CPU FP64 oracle of OmniTrack's matching and update phases (Sec. V-A).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the
smoke check and the benchmark's CPU-baseline leg use it; the product never
imports it.  Plain NumPy/SciPy, written from the definitions:

- matching score: intersection over union of two axis-aligned boxes
  (x0, y0, x1, y1), area = max(0, x1 - x0) * max(0, y1 - y0);
- matching: the globally optimal one-to-one assignment of predicted scene
  objects to detections maximising the summed IoU (Kuhn 1955), taken by
  SciPy's linear_sum_assignment as the library step; only pairs with IoU at
  least `iou_min` may match;
- update: an unmatched scene object is flagged lost and takes no further
  part; an unmatched detection becomes a new scene object.  A matched object
  takes its detection's box.
"""
from __future__ import annotations

import numpy as np
import scipy.optimize


def box_area(b) -> float:
    return max(0.0, float(b[2]) - float(b[0])) * max(0.0, float(b[3]) - float(b[1]))


def iou(a, b) -> float:
    """IoU of two boxes; 0 when the union has no area."""
    ix = max(0.0, min(float(a[2]), float(b[2])) - max(float(a[0]), float(b[0])))
    iy = max(0.0, min(float(a[3]), float(b[3])) - max(float(a[1]), float(b[1])))
    inter = ix * iy
    union = box_area(a) + box_area(b) - inter
    return inter / union if union > 0.0 else 0.0


def iou_matrix(S, D, active=None) -> np.ndarray:
    """(m, k) FP64 IoU of every scene box S[i] with every detection D[j];
    rows of inactive (lost) objects are 0."""
    S = np.asarray(S, np.float64).reshape(-1, 4)
    D = np.asarray(D, np.float64).reshape(-1, 4)
    out = np.zeros((S.shape[0], D.shape[0]), np.float64)
    for i in range(S.shape[0]):
        if active is not None and not active[i]:
            continue
        for j in range(D.shape[0]):
            out[i, j] = iou(S[i], D[j])
    return out


def assign(iou_m, iou_min: float):
    """Optimal matching: (s2d (m,) int32, d2s (k,) int32, score float).
    s2d[i] = j when object i is matched to detection j, else -1; score is
    the summed IoU of the matched pairs."""
    w = np.asarray(iou_m, np.float64)
    m, k = w.shape
    s2d = np.full(m, -1, np.int32)
    d2s = np.full(k, -1, np.int32)
    if m == 0 or k == 0:
        return s2d, d2s, 0.0
    gain = np.where(w >= iou_min, w, 0.0)
    rows, cols = scipy.optimize.linear_sum_assignment(gain, maximize=True)
    score = 0.0
    for r, c in zip(rows, cols):
        if w[r, c] >= iou_min:
            s2d[r] = c
            d2s[c] = r
            score += w[r, c]
    return s2d, d2s, score


def track_update(boxes, ids, lost, det, s2d, d2s, next_id: int):
    """The update phase: returns (boxes (m', 4), ids (m',), lost (m',),
    next_id).  Existing objects keep their order; new ones follow in
    detection order with ids next_id, next_id + 1, ..."""
    boxes = [np.asarray(b, np.float64) for b in np.asarray(boxes, np.float64).reshape(-1, 4)]
    ids = [int(v) for v in ids]
    lost = [int(v) for v in lost]
    det = np.asarray(det, np.float64).reshape(-1, 4)
    for i in range(len(boxes)):
        if lost[i]:
            continue
        if s2d[i] >= 0:
            boxes[i] = det[s2d[i]].copy()
        else:
            lost[i] = 1
    for j in range(det.shape[0]):
        if d2s[j] < 0:
            boxes.append(det[j].copy())
            ids.append(next_id)
            lost.append(0)
            next_id += 1
    return (np.asarray(boxes, np.float64).reshape(-1, 4), np.asarray(ids, np.int32),
            np.asarray(lost, np.uint8), next_id)
