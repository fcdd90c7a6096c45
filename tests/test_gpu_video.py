"""One video stream tracked frame by frame at its working level, with and
without the prefetch of the next frame's preprocessing (Sec. V-B), the
longest-first order from the previous pair's iteration counts and the
Scharr planes built with each frame's pyramid: all give
identical boxes and counts on every frame (same kernels, same inputs, only
the streams and the order of the points differ), and the frames right after
a re-seed match the oracle's tracker and box update at the working level
(counts equal, every box within 0.01 px)."""
import numpy as np
import pytest

import oracle
import parity_log
from paper_1910_06017_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_06017_amd import ops, video
    ops.lib()
    s = synth.served_streams(seed=91, nstreams=1, nframes=12, npts_range=(3000, 3000),
                             nbox_range=(6, 6), resolutions=((2560, 1280),))[0]
    frames = []
    for f in s.frames:
        t = torch.empty(f.shape, dtype=torch.uint8, pin_memory=True)
        t.copy_(torch.from_numpy(f))
        frames.append(t)
    seeds = {k: s.seed_points(k, np.random.default_rng(500 + k)) for k in (0, 10)}
    return ops, video, s, frames, seeds


def test_prefetch_and_order_give_identical_results(env):
    ops, video, s, frames, seeds = env
    base = ops.working_level(s.W, s.H)
    assert base == 1
    runs = []
    for pf, order, grads in ((False, False, False), (True, False, False), (True, True, False),
                             (True, False, True)):
        trk = video.VideoTracker(s.W, s.H, levels=4, base_level=base, n_max=4000, m_max=16,
                                 prefetch=pf, order=order, grads=grads)
        runs.append(trk.track(frames, seeds))
    assert len(runs[0]) == len(frames) - 1
    for other in runs[1:]:
        for (b0, c0), (b1, c1) in zip(runs[0], other):
            assert np.array_equal(b0, b1) and np.array_equal(c0, c1)


def test_reseeded_frames_match_oracle(env):
    ops, video, s, frames, seeds = env
    base = ops.working_level(s.W, s.H)
    trk = video.VideoTracker(s.W, s.H, levels=4, base_level=base, n_max=4000, m_max=16)
    res = trk.track(frames, seeds)
    worst, same_n, boxes_n = 0.0, 0, 0
    for k in seeds:
        if k + 1 >= len(frames):
            continue
        pts, bid, bx = seeds[k]
        o = oracle.lk_track_working(s.frames[k], s.frames[k + 1], pts, base, 21, 4, 30,
                                    float(np.float32(0.01)))
        ob, oc = oracle.box_update(bx, bid, pts, o.next_pts, o.status)
        gb, gc = res[k]            # predicted for frame k + 1
        same = gc == oc
        same_n += same.sum()
        boxes_n += len(oc)
        worst = max(worst, float(np.abs(gb[same] - ob[same]).max()))
    parity_log.record(f"video 2560x1280 at working level {base}, prefetch: {boxes_n} boxes "
                      f"after re-seeds, counts equal {same_n / boxes_n:.4f}, max corner "
                      f"difference {worst:.2e} px")
    assert same_n == boxes_n
    assert worst <= 0.01
