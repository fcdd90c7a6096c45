"""CPU oracle of the working-level choice of OmniTrack's preprocessing phase
(Sec. V-A): the frame is reduced by the Gaussian pyramid and motion is
computed at a level chosen from the resolution, so that large frames are
not processed at full size.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper names the
idea but no rule; the rule here is the smallest level whose width is at
most `max_width` (1280 by default: SD stays at level 0, 2560-wide frames
go to level 1, 3840-wide to level 2).
"""
from __future__ import annotations

import numpy as np


def working_level(W: int, H: int, max_width: int = 1280) -> int:
    """Smallest level l with w_l <= max_width, w_0 = W, w_l = ceil(w_{l-1} / 2)."""
    if W < 1 or H < 1 or max_width < 1:
        return -1
    level, w = 0, W
    while w > max_width:
        w = -(-w // 2)
        level += 1
    return level


def lk_track_working(frame0, frame1, pts, base: int, win: int = 21, levels: int = 3,
                     iters: int = 30, eps: float = 0.01, min_eig: float | None = None):
    """Track at working level `base`: the pyramids' levels base .. base+levels-1
    form the tracked pyramid, points enter divided by 2^base and leave
    multiplied by it (both exact in binary floating point).  Returns the
    oracle's LK result with next_pts in level-0 pixels."""
    import oracle
    P = oracle.pyramid(frame0, base + levels)[base:]
    Q = oracle.pyramid(frame1, base + levels)[base:]
    s = np.float32(2.0 ** -base)
    kw = {} if min_eig is None else {"min_eig": min_eig}
    r = oracle.lk_track_pyr(P, Q, np.asarray(pts, np.float32) * s, win, levels, iters, eps, **kw)
    r.next_pts = r.next_pts * 2.0 ** base
    return r
