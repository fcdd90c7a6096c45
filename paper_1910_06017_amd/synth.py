"""Seeded synthetic video workloads for the tracking path.

Everything here *makes inputs*: textured grayscale frames, point grids,
per-point box ids, boxes, and the true motion of every point.  It holds none
of the tracker's arithmetic (no pyramid, no gradients, no interpolation of a
frame, no flow, no medians), so the CPU oracle and the HIP path can both take
their inputs from it without sharing any part of the method.

The paper's own videos and datasets are not available, so these scenes stand
in for them at the paper's standard-definition size (720x576, Sec. VI) and at
720p / 1080p.  Every random number comes from ``numpy.random.default_rng``
(PCG64) with an explicit seed, so a workload is a pure function of its seed.

Surfaces are sums of 2-D plane waves and isotropic Gaussian blobs.  Such a sum
stays in the same family under a similarity transform (scale, rotation,
translation), so a moved surface is rendered exactly from transformed
parameters, and every pixel block is one dense product of a (rows x K) by a
(K x cols) matrix.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "Texture", "Rect", "Scene", "Workload", "Stream",
    "random_texture", "render_scene", "grid_points",
    "shifted_pair", "boxes_pair", "sd_shift_workload", "sd_boxes_workload",
    "hd_boxes_workload", "batched_streams", "served_streams",
    "RESOLUTIONS",
]

RESOLUTIONS = ((720, 576), (1280, 720), (1920, 1080))


# --------------------------------------------------------------------------
# Surfaces
# --------------------------------------------------------------------------
@dataclass
class Texture:
    """f(p) = sum_k A_k sin(w_k . p + phi_k) + sum_j a_j exp(-|p - c_j|^2 / (2 s_j^2))."""

    amp: np.ndarray      # (K,)
    omega: np.ndarray    # (K, 2) radians per pixel
    phase: np.ndarray    # (K,)
    bamp: np.ndarray     # (B,)
    bcen: np.ndarray     # (B, 2)
    bsig: np.ndarray     # (B,)

    def moved(self, scale: float, theta: float, centre, t) -> "Texture":
        """Texture g with g(M p) = f(p) for M p = c + t + scale * R(theta) (p - c)."""
        c = np.asarray(centre, np.float64)
        t = np.asarray(t, np.float64)
        co, si = math.cos(theta), math.sin(theta)
        rot = np.array([[co, -si], [si, co]])
        # f(M^-1 q): w . (R^T (q - c - t) / s + c) = (R w / s) . (q - c - t) + w . c
        om2 = (self.omega @ rot.T) / scale
        ph2 = self.phase + self.omega @ c - om2 @ (c + t)
        cen2 = c + t + scale * ((self.bcen - c) @ rot.T)
        return Texture(self.amp.copy(), om2, ph2, self.bamp.copy(), cen2,
                       self.bsig * scale)

    def render(self, x0: int, y0: int, w: int, h: int) -> np.ndarray:
        """Values at integer pixels x0..x0+w-1, y0..y0+h-1 as an (h, w) float64 array."""
        xs = x0 + np.arange(w, dtype=np.float64)
        ys = y0 + np.arange(h, dtype=np.float64)
        ax = self.omega[:, 0:1] * xs[None, :] + self.phase[:, None]      # (K, w)
        by = ys[:, None] * self.omega[None, :, 1]                          # (h, K)
        left = [np.cos(by) * self.amp, np.sin(by) * self.amp]
        right = [np.sin(ax), np.cos(ax)]
        if self.bamp.size:
            inv = 1.0 / (2.0 * self.bsig ** 2)
            gx = np.exp(-((xs[None, :] - self.bcen[:, 0:1]) ** 2) * inv[:, None])
            gy = np.exp(-((ys[:, None] - self.bcen[None, :, 1]) ** 2) * inv[None, :])
            left.append(gy * self.bamp)
            right.append(gx)
        return np.concatenate(left, axis=1) @ np.concatenate(right, axis=0)


def random_texture(rng: np.random.Generator, n_waves: int, n_blobs: int,
                   extent, period=(8.0, 64.0), sigma=(2.0, 10.0)) -> Texture:
    """Random plane waves (amplitude U[0.5,1], log-uniform period, orientation
    U[0,pi), phase U[0,2pi)) plus blobs centred uniformly over `extent`
    = (x0, y0, x1, y1) with sigma U[sigma] and signed amplitude U[-1,1]."""
    amp = rng.uniform(0.5, 1.0, n_waves)
    per = np.exp(rng.uniform(math.log(period[0]), math.log(period[1]), n_waves))
    ang = rng.uniform(0.0, math.pi, n_waves)
    phase = rng.uniform(0.0, 2.0 * math.pi, n_waves)
    k = 2.0 * math.pi / per
    omega = np.stack([k * np.cos(ang), k * np.sin(ang)], axis=1)
    x0, y0, x1, y1 = extent
    bcen = np.stack([rng.uniform(x0, x1, n_blobs), rng.uniform(y0, y1, n_blobs)], axis=1)
    bsig = rng.uniform(sigma[0], sigma[1], n_blobs)
    bamp = rng.uniform(-1.0, 1.0, n_blobs)
    return Texture(amp, omega, phase, bamp, bcen, bsig)


@dataclass
class Rect:
    """A textured rectangle, axis-aligned at frame 0, moving by a similarity.

    ``poses[k] = (scale, theta, tx, ty)`` maps frame-0 positions p to frame-k
    positions c + t + scale R(theta) (p - c), with c the frame-0 centre.
    """

    cx: float
    cy: float
    hw: float
    hh: float
    tex: Texture
    lo: float            # frame-0 texture minimum over the rectangle (for scaling)
    hi: float
    poses: list

    def transform(self, k: int):
        s, th, tx, ty = self.poses[k]
        return s, th, (self.cx, self.cy), (tx, ty)

    def map_points(self, k: int, p: np.ndarray) -> np.ndarray:
        s, th, c, t = self.transform(k)
        co, si = math.cos(th), math.sin(th)
        d = p - np.asarray(c)
        return np.stack([c[0] + t[0] + s * (co * d[:, 0] - si * d[:, 1]),
                         c[1] + t[1] + s * (si * d[:, 0] + co * d[:, 1])], axis=1)

    def inside(self, k: int, p: np.ndarray) -> np.ndarray:
        s, th, c, t = self.transform(k)
        co, si = math.cos(th), math.sin(th)
        d = p - np.asarray(c) - np.asarray(t)
        lx = (co * d[..., 0] + si * d[..., 1]) / s
        ly = (-si * d[..., 0] + co * d[..., 1]) / s
        return (np.abs(lx) <= self.hw) & (np.abs(ly) <= self.hh)

    def bbox(self, k: int):
        """Axis-aligned bounds (x0, y0, x1, y1) of the rectangle in frame k."""
        s, th, c, t = self.transform(k)
        ex = s * (abs(math.cos(th)) * self.hw + abs(math.sin(th)) * self.hh)
        ey = s * (abs(math.sin(th)) * self.hw + abs(math.cos(th)) * self.hh)
        mx, my = c[0] + t[0], c[1] + t[1]
        return (mx - ex, my - ey, mx + ex, my + ey)


@dataclass
class Scene:
    W: int
    H: int
    bg: Texture
    bg_lo: float
    bg_hi: float
    rects: list = field(default_factory=list)
    noise: float = 0.0


def _to_unit(v, lo, hi):
    return (v - lo) * (255.0 / max(hi - lo, 1e-12))


def render_scene(scene: Scene, k: int, rng: np.random.Generator | None) -> np.ndarray:
    """Frame k of a scene: static background, rectangles painted in index
    order, optional N(0, noise) per frame, clipped and rounded to uint8."""
    W, H = scene.W, scene.H
    img = _to_unit(scene.bg.render(0, 0, W, H), scene.bg_lo, scene.bg_hi)
    for r in scene.rects:
        x0, y0, x1, y1 = r.bbox(k)
        ix0, iy0 = max(0, int(math.floor(x0)) - 1), max(0, int(math.floor(y0)) - 1)
        ix1, iy1 = min(W - 1, int(math.ceil(x1)) + 1), min(H - 1, int(math.ceil(y1)) + 1)
        if ix1 < ix0 or iy1 < iy0:
            continue
        s, th, c, t = r.transform(k)
        tex = r.tex.moved(s, th, c, t)
        blk = _to_unit(tex.render(ix0, iy0, ix1 - ix0 + 1, iy1 - iy0 + 1), r.lo, r.hi)
        gx, gy = np.meshgrid(np.arange(ix0, ix1 + 1, dtype=np.float64),
                             np.arange(iy0, iy1 + 1, dtype=np.float64))
        m = r.inside(k, np.stack([gx, gy], axis=-1))
        sub = img[iy0:iy1 + 1, ix0:ix1 + 1]
        sub[m] = blk[m]
    if scene.noise > 0 and rng is not None:
        img = img + rng.normal(0.0, scene.noise, img.shape)
    return np.floor(np.clip(img, 0.0, 255.0) + 0.5).astype(np.uint8)


def grid_points(box, nx: int, ny: int, count: int | None = None) -> np.ndarray:
    """Centres of an nx x ny grid of cells covering box = (x0, y0, x1, y1), row-major."""
    x0, y0, x1, y1 = box
    gx = x0 + (np.arange(nx) + 0.5) * (x1 - x0) / nx
    gy = y0 + (np.arange(ny) + 0.5) * (y1 - y0) / ny
    X, Y = np.meshgrid(gx, gy)
    p = np.stack([X.ravel(), Y.ravel()], axis=1)
    return p if count is None else p[:count]


def _grid_for_count(box, n: int) -> np.ndarray:
    x0, y0, x1, y1 = box
    ar = max(x1 - x0, 1e-6) / max(y1 - y0, 1e-6)
    nx = max(1, int(math.ceil(math.sqrt(n * ar))))
    ny = max(1, int(math.ceil(n / nx)))
    return grid_points(box, nx, ny, n)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    """One frame pair with points.  Frames are (H, W) uint8, row-major."""

    name: str
    frame0: np.ndarray
    frame1: np.ndarray
    pts: np.ndarray          # (n, 2) float32, level-0 pixels, centres at integers
    truth: np.ndarray        # (n, 2) float64 true displacement of each point
    box_id: np.ndarray       # (n,) int32, -1 = no box
    boxes: np.ndarray        # (m, 4) float32 (x0, y0, x1, y1) at frame 0
    boxes_next: np.ndarray   # (m, 4) float64 true boxes at frame 1
    win: int = 21
    levels: int = 4
    iters: int = 30
    eps: float = 0.01

    @property
    def W(self):
        return self.frame0.shape[1]

    @property
    def H(self):
        return self.frame0.shape[0]

    @property
    def n(self):
        return self.pts.shape[0]


def _place_rect(rng, W, H, side, trans, scale_rng, rot_deg, margin=12.0, tries=200):
    """Draw a rectangle and its motion so it stays `margin` px inside both frames."""
    for _ in range(tries):
        w = rng.uniform(*side)
        h = rng.uniform(*side)
        hw, hh = w / 2.0, h / 2.0
        tx, ty = rng.uniform(-trans, trans, 2)
        s = rng.uniform(*scale_rng) if scale_rng else 1.0
        th = math.radians(rng.uniform(-rot_deg, rot_deg)) if rot_deg else 0.0
        ex = s * (abs(math.cos(th)) * hw + abs(math.sin(th)) * hh)
        ey = s * (abs(math.sin(th)) * hw + abs(math.cos(th)) * hh)
        lox = max(margin + hw, margin + ex - tx)
        hix = min(W - 1 - margin - hw, W - 1 - margin - ex - tx)
        loy = max(margin + hh, margin + ey - ty)
        hiy = min(H - 1 - margin - hh, H - 1 - margin - ey - ty)
        if lox <= hix and loy <= hiy:
            return rng.uniform(lox, hix), rng.uniform(loy, hiy), hw, hh, (s, th, tx, ty)
    raise RuntimeError("could not place a rectangle")


def _make_rect(rng, cx, cy, hw, hh, poses, n_waves=24):
    area = 4.0 * hw * hh
    n_blobs = max(8, int(round(200.0 * area / (720.0 * 576.0))))
    tex = random_texture(rng, n_waves, n_blobs, (cx - hw, cy - hh, cx + hw, cy + hh))
    ix0, iy0 = int(math.ceil(cx - hw)), int(math.ceil(cy - hh))
    ix1, iy1 = int(math.floor(cx + hw)), int(math.floor(cy + hh))
    v = tex.render(ix0, iy0, max(1, ix1 - ix0 + 1), max(1, iy1 - iy0 + 1))
    return Rect(cx, cy, hw, hh, tex, float(v.min()), float(v.max()), poses)


def _background(rng, W, H, pad=16):
    tex = random_texture(rng, 64, 200, (-pad, -pad, W + pad, H + pad))
    v = tex.render(-pad, -pad, W + 2 * pad, H + 2 * pad)
    return tex, float(v.min()), float(v.max())


def _truth(scene: Scene, pts: np.ndarray, k0: int, k1: int) -> np.ndarray:
    """Motion of the topmost surface under each point from frame k0 to k1."""
    d = np.zeros_like(pts, dtype=np.float64)
    done = np.zeros(len(pts), bool)
    for r in reversed(scene.rects):
        m = ~done & r.inside(k0, pts)
        if m.any():
            # frame-k0 position -> frame-0 position -> frame-k1 position
            s, th, c, t = r.transform(k0)
            co, si = math.cos(th), math.sin(th)
            q = pts[m] - np.asarray(c) - np.asarray(t)
            p0 = np.stack([c[0] + (co * q[:, 0] + si * q[:, 1]) / s,
                           c[1] + (-si * q[:, 0] + co * q[:, 1]) / s], axis=1)
            d[m] = r.map_points(k1, p0) - pts[m]
            done |= m
    return d


def shifted_pair(seed: int, W: int = 720, H: int = 576, shift=None,
                 mode: str = "bilinear", pad: int = 16, max_shift: float = 3.0):
    """Texture frame and a copy moved by one global sub-pixel shift (dx, dy).

    mode "bilinear": frame1 = FP64 bilinear resampling of frame 0's padded
    canvas at p - d (the canvas is wide enough that it never reads outside).
    mode "analytic": frame1 is the texture rendered exactly at p - d.
    Returns (frame0, frame1, (dx, dy)).
    """
    rng = np.random.default_rng(seed)
    tex, lo, hi = _background(rng, W, H, pad)
    if shift is None:
        shift = rng.uniform(-max_shift, max_shift, 2)
    dx, dy = float(shift[0]), float(shift[1])
    canvas = _to_unit(tex.render(-pad, -pad, W + 2 * pad, H + 2 * pad), lo, hi)
    f0 = np.floor(np.clip(canvas[pad:pad + H, pad:pad + W], 0, 255) + 0.5).astype(np.uint8)
    if mode == "analytic":
        mt = tex.moved(1.0, 0.0, (0.0, 0.0), (dx, dy))
        c1 = _to_unit(mt.render(0, 0, W, H), lo, hi)
    elif mode == "bilinear":
        assert abs(dx) < pad - 1 and abs(dy) < pad - 1
        sx, sy = -dx, -dy
        ix, iy = int(math.floor(sx)), int(math.floor(sy))
        ax, ay = sx - ix, sy - iy
        r0, c0 = pad + iy, pad + ix
        A = canvas[r0:r0 + H, c0:c0 + W]
        B = canvas[r0:r0 + H, c0 + 1:c0 + 1 + W]
        C = canvas[r0 + 1:r0 + 1 + H, c0:c0 + W]
        D = canvas[r0 + 1:r0 + 1 + H, c0 + 1:c0 + 1 + W]
        c1 = (1 - ax) * (1 - ay) * A + ax * (1 - ay) * B + (1 - ax) * ay * C + ax * ay * D
    else:
        raise ValueError(mode)
    f1 = np.floor(np.clip(c1, 0, 255) + 0.5).astype(np.uint8)
    return f0, f1, (dx, dy)


def sd_shift_workload(seed: int = 101, mode: str = "bilinear") -> Workload:
    """720x576 texture pair under one global sub-pixel shift d ~ U[-3,3]^2,
    1024 points on a 32x32 grid at ((i+0.5)*22.5, (j+0.5)*18); window 21,
    3 levels, 30 iterations, eps 0.01."""
    f0, f1, (dx, dy) = shifted_pair(seed, 720, 576, mode=mode)
    i = np.arange(32)
    X, Y = np.meshgrid((i + 0.5) * 22.5, (i + 0.5) * 18.0)
    pts = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float32)
    truth = np.tile(np.array([[dx, dy]]), (len(pts), 1))
    return Workload("sd_shift", f0, f1, pts, truth, np.full(len(pts), -1, np.int32),
                    np.zeros((0, 4), np.float32), np.zeros((0, 4)), 21, 3, 30, 0.01)


def _boxes_scene(rng, W, H, nrect, side, trans, scale_rng, rot_deg, noise, nframes=2,
                 poses_fn=None):
    bg, lo, hi = _background(rng, W, H)
    scene = Scene(W, H, bg, lo, hi, noise=noise)
    for _ in range(nrect):
        cx, cy, hw, hh, pose = _place_rect(rng, W, H, side, trans, scale_rng, rot_deg)
        poses = [(1.0, 0.0, 0.0, 0.0), pose] if poses_fn is None else poses_fn(rng, pose)
        scene.rects.append(_make_rect(rng, cx, cy, hw, hh, poses))
    return scene


def boxes_pair(seed: int, W: int, H: int, nrect: int, side, trans, scale_rng, rot_deg,
               noise: float, pts_per_box, name: str, levels: int,
               grid: int | None = None) -> Workload:
    """Static textured background plus `nrect` textured rectangles, each moving
    by its own similarity; per-frame Gaussian noise; grid points in every box."""
    rng = np.random.default_rng(seed)
    scene = _boxes_scene(rng, W, H, nrect, side, trans, scale_rng, rot_deg, noise)
    nrng = np.random.default_rng(seed + 1_000_003)
    f0 = render_scene(scene, 0, nrng)
    f1 = render_scene(scene, 1, nrng)
    pts, bid, boxes, boxes1 = [], [], [], []
    for b, r in enumerate(scene.rects):
        box = r.bbox(0)
        boxes.append(box)
        boxes1.append(r.bbox(1))
        n_b = pts_per_box[b] if not np.isscalar(pts_per_box) else pts_per_box
        p = grid_points(box, grid, grid) if grid else _grid_for_count(box, int(n_b))
        pts.append(p)
        bid.append(np.full(len(p), b, np.int32))
    pts = np.concatenate(pts).astype(np.float32)
    truth = _truth(scene, pts.astype(np.float64), 0, 1)
    return Workload(name, f0, f1, pts, truth, np.concatenate(bid),
                    np.asarray(boxes, np.float32), np.asarray(boxes1, np.float64),
                    21, levels, 30, 0.01)


def sd_boxes_workload(seed: int = 202) -> Workload:
    """720x576, 20 rectangles (sides U[40,160], translation U[-20,20]^2, scale
    U[0.95,1.05]), noise sigma 2, 400 points per box on a 20x20 grid; window
    21, 4 levels, 30 iterations."""
    return boxes_pair(seed, 720, 576, 20, (40.0, 160.0), 20.0, (0.95, 1.05), 0.0, 2.0,
                      400, "sd_boxes", 4, grid=20)


def hd_boxes_workload(seed: int = 303) -> Workload:
    """1920x1080, 16 rectangles (sides U[80,400], translation U[-40,40]^2,
    rotation U[-3,3] deg), noise sigma 3, 900 points per box on a 30x30 grid;
    window 21, 5 levels, 30 iterations."""
    return boxes_pair(seed, 1920, 1080, 16, (80.0, 400.0), 40.0, None, 3.0, 3.0,
                      900, "hd_boxes", 5, grid=30)


def _stream_params(W):
    """Motion recipe by resolution: SD as the 720x576 box scene, larger sizes as
    the 1080p scene scaled by W/1920."""
    if W == 720:
        return dict(side=(40.0, 160.0), trans=20.0, scale_rng=(0.95, 1.05), rot_deg=0.0,
                    noise=2.0, levels=4)
    k = W / 1920.0
    return dict(side=(80.0 * k, 400.0 * k), trans=40.0 * k, scale_rng=None, rot_deg=3.0,
                noise=3.0, levels=4 if W <= 1280 else 5)


def batched_streams(seed: int = 404, nstreams: int = 32, npts_range=(500, 20000),
                    nbox_range=(4, 30), resolutions=RESOLUTIONS) -> list:
    """Independent streams: resolution uniform over `resolutions`, box count
    uniform in nbox_range, points log-uniform in npts_range split evenly over
    the boxes.  Returns a list of Workload (one frame pair each)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(nstreams):
        W, H = resolutions[int(rng.integers(len(resolutions)))]
        m = int(rng.integers(nbox_range[0], nbox_range[1] + 1))
        n = int(round(math.exp(rng.uniform(math.log(npts_range[0]), math.log(npts_range[1])))))
        per = [n // m + (1 if b < n % m else 0) for b in range(m)]
        prm = _stream_params(W)
        sub = int(rng.integers(1 << 31))
        wl = boxes_pair(sub, W, H, m, prm["side"], prm["trans"], prm["scale_rng"],
                        prm["rot_deg"], prm["noise"], per, f"stream{s}", prm["levels"])
        out.append(wl)
    return out


@dataclass
class Stream:
    """A simulated video stream: a cycle of frames plus the true boxes of every
    frame, for the serving loop.  Frame k pairs with frame k-1."""

    sid: int
    W: int
    H: int
    levels: int
    frames: list            # (H, W) uint8 per frame of the cycle
    boxes: np.ndarray       # (nframes, m, 4) float64 true boxes per frame
    pts_per_box: list
    fps: float = 25.0

    def seed_points(self, k: int, rng: np.random.Generator, jitter: float = 1.0):
        """Synthetic 'detections' at frame k: true boxes plus N(0, jitter) px,
        and grid points inside them.  Returns (pts float32, box_id int32, boxes float32)."""
        bx = self.boxes[k % len(self.frames)] + rng.normal(0.0, jitter, self.boxes.shape[1:])
        bx[:, 2] = np.maximum(bx[:, 2], bx[:, 0] + 2.0)
        bx[:, 3] = np.maximum(bx[:, 3], bx[:, 1] + 2.0)
        pts, bid = [], []
        for b in range(bx.shape[0]):
            p = _grid_for_count(tuple(bx[b]), self.pts_per_box[b])
            pts.append(p)
            bid.append(np.full(len(p), b, np.int32))
        pts = np.clip(np.concatenate(pts), 0.0, [self.W - 1.0, self.H - 1.0])
        return pts.astype(np.float32), np.concatenate(bid), bx.astype(np.float32)


def detections(true_boxes, rng: np.random.Generator, W: int, H: int, jitter: float = 1.0,
               miss: float = 0.1, extra: int = 2, side=(30.0, 120.0)) -> np.ndarray:
    """Synthetic detector output for one frame: each true box, with
    probability 1 - miss, plus N(0, jitter) px per coordinate; then `extra`
    boxes of random size at random places (objects entering the scene), all
    in random order.  (k, 4) float32 (x0, y0, x1, y1)."""
    tb = np.asarray(true_boxes, np.float64).reshape(-1, 4)
    keep = rng.uniform(size=len(tb)) >= miss
    d = tb[keep] + rng.normal(0.0, jitter, (int(keep.sum()), 4))
    d[:, 2] = np.maximum(d[:, 2], d[:, 0] + 2.0)
    d[:, 3] = np.maximum(d[:, 3], d[:, 1] + 2.0)
    wh = rng.uniform(side[0], side[1], (extra, 2))
    xy = rng.uniform([0.0, 0.0], [W - side[1], H - side[1]], (extra, 2))
    d = np.concatenate([d, np.concatenate([xy, xy + wh], axis=1)])
    return d[rng.permutation(len(d))].astype(np.float32)


def served_streams(seed: int = 505, nstreams: int = 64, nframes: int = 20,
                   npts_range=(500, 20000), nbox_range=(4, 30),
                   resolutions=RESOLUTIONS) -> list:
    """Streams for the serving loop.  Each rectangle oscillates (translation
    amplitude as the batched recipe, rotation/scale likewise) with period
    `nframes` between its frame-0 placement and a drawn pose, so the frame
    cycle wraps without a jump."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(nstreams):
        W, H = resolutions[int(rng.integers(len(resolutions)))]
        m = int(rng.integers(nbox_range[0], nbox_range[1] + 1))
        n = int(round(math.exp(rng.uniform(math.log(npts_range[0]), math.log(npts_range[1])))))
        per = [n // m + (1 if b < n % m else 0) for b in range(m)]
        prm = _stream_params(W)
        srng = np.random.default_rng(int(rng.integers(1 << 31)))

        def poses_fn(r, pose, F=nframes):
            # lam in [0, 1]: every pose lies between the identity and the drawn
            # pose, both of which keep the rectangle inside the frame.
            s1, th1, tx1, ty1 = pose
            psi = r.uniform(0, 2 * math.pi)
            out_p = []
            for k in range(F):
                lam = 0.5 * (1.0 - math.cos(2 * math.pi * k / F + psi))
                out_p.append((1.0 + (s1 - 1.0) * lam, th1 * lam, tx1 * lam, ty1 * lam))
            return out_p

        scene = _boxes_scene(srng, W, H, m, prm["side"], prm["trans"], prm["scale_rng"],
                             prm["rot_deg"], prm["noise"], poses_fn=poses_fn)
        nrng = np.random.default_rng(int(srng.integers(1 << 31)))
        frames = [render_scene(scene, k, nrng) for k in range(nframes)]
        boxes = np.array([[r.bbox(k) for r in scene.rects] for k in range(nframes)])
        out.append(Stream(s, W, H, prm["levels"], frames, boxes, per))
    return out


def similarity_box_points(seed: int, counts, outlier_frac: float = 0.1, lost_frac: float = 0.05,
                          dup: bool = False, extra_ids: bool = True):
    """Point sets for the scaled box update: box b gets counts[b] points drawn
    uniformly in a random box, moved by a random similarity (scale 0.9-1.1
    about the box centre, shift up to 30 px) plus 0.05 px noise, with a
    fraction of outliers (25 px noise) and of lost points (status 0); ids are
    interleaved in random order, and a few points carry ids of no box.  With
    dup every point of a box has a coincident twin.  Returns (boxes (m, 4),
    box_id (n,), pts (n, 2), next_pts (n, 2), status (n,))."""
    rng = np.random.default_rng(seed)
    m = len(counts)
    boxes, P, Q, ids = [], [], [], []
    for b, c in enumerate(counts):
        w, h = rng.uniform(20, 400, 2)
        x0, y0 = rng.uniform(0, 1500), rng.uniform(0, 700)
        boxes.append([x0, y0, x0 + w, y0 + h])
        s = rng.uniform(0.9, 1.1)
        t = rng.uniform(-30, 30, 2)
        p = rng.uniform([x0, y0], [x0 + w, y0 + h], (c, 2))
        if dup and c > 4:
            p[c // 2:] = p[: c - c // 2]
        cen = np.array([x0 + w / 2, y0 + h / 2])
        q = cen + t + s * (p - cen) + rng.normal(0, 0.05, (c, 2))
        bad = rng.random(c) < outlier_frac
        q[bad] += rng.normal(0, 25, (bad.sum(), 2))
        P.append(p)
        Q.append(q)
        ids.append(np.full(c, b, np.int32))
    P = np.concatenate(P) if P else np.zeros((0, 2))
    Q = np.concatenate(Q) if Q else np.zeros((0, 2))
    ids = np.concatenate(ids) if ids else np.zeros(0, np.int32)
    if extra_ids:
        k = max(1, len(ids) // 50)
        P = np.concatenate([P, rng.uniform(0, 1000, (k, 2))])
        Q = np.concatenate([Q, rng.uniform(0, 1000, (k, 2))])
        ids = np.concatenate([ids, rng.choice([-1, m, m + 7], k).astype(np.int32)])
    st = (rng.random(len(ids)) >= lost_frac).astype(np.uint8)
    perm = rng.permutation(len(ids))
    return (np.asarray(boxes, np.float32), ids[perm].astype(np.int32), P[perm].astype(np.float32),
            Q[perm].astype(np.float32), st[perm])
