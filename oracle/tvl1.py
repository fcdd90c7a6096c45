"""CPU FP64 oracle of the dense variant of the motion features: TV-L1 optical
flow with a Huber-smoothed total variation, solved by projected gradient
steps on the dual variable, on structure-texture decomposed inputs
(Sec. IV), and the per-box mean of the dense field (Sec. V-A prediction).

TEST INFRASTRUCTURE ONLY (see the package docstring).  NumPy, whole-image
array operations in FP64, following the steps in order:

- images are the uint8 pyramid levels (the same pyramid as the sparse
  path) scaled to [0, 1];
- structure-texture split of every level: structure = the minimiser of
  TV(s) + |s - f|^2 / (2 theta_s) by Chambolle's dual iteration (2004),
  texture = f - alpha * structure;
- coarse-to-fine over the levels, `warps` linearisations per level and
  `iters` iterations per linearisation of: v from the pointwise L1 data
  step (soft thresholding along the image gradient), u = v + theta div p,
  p = projection onto |p| <= 1 of (p + (tau/theta) grad u) / (1 + tau eps /
  theta), separately for both flow components (Zach, Pock & Bischof 2007;
  Huber smoothing as in Werlberger et al. 2009);
- grad: forward differences, 0 on the last column / row; div = -grad^T
  (Chambolle 2004);
- warping: the second texture and its central-difference gradient (clamped
  indices) sampled bilinearly at x + u0 with clamp-to-edge;
- a coarse flow enters the next finer level as 2 * bilinear(u, x / 2); the
  dual variable restarts at 0 on every level.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class TvL1Params:
    levels: int = 5
    warps: int = 5
    iters: int = 30
    lam: float = 40.0        # data weight, textures on the [0, 1] scale (0.16 on 0..255)
    theta: float = 0.3       # coupling of u and v
    tau: float = 0.25        # dual step
    eps: float = 0.01        # Huber smoothing of the total variation
    alpha: float = 0.95      # texture = f - alpha * structure
    theta_s: float = 0.1     # structure (ROF) fidelity weight
    tau_s: float = 0.125     # structure dual step
    iters_s: int = 50        # structure iterations


def grad(u):
    """Forward differences; 0 on the last column (x) and the last row (y)."""
    gx = np.zeros_like(u)
    gy = np.zeros_like(u)
    gx[:, :-1] = u[:, 1:] - u[:, :-1]
    gy[:-1, :] = u[1:, :] - u[:-1, :]
    return gx, gy


def div(px, py):
    """Negative adjoint of grad: backward differences of p with p taken as 0
    on the last column (x) / row (y) and before the first."""
    qx = px.copy()
    qx[:, -1] = 0.0
    qy = py.copy()
    qy[-1, :] = 0.0
    d = qx + qy
    d[:, 1:] -= qx[:, :-1]
    d[1:, :] -= qy[:-1, :]
    return d


def rof(f, theta: float, tau: float, iters: int):
    """Structure part: argmin_s TV(s) + |s - f|^2 / (2 theta), Chambolle's
    dual fixed point p <- (p + tau grad(div p - f/theta)) /
    (1 + tau |grad(div p - f/theta)|), s = f - theta div p."""
    px = np.zeros_like(f)
    py = np.zeros_like(f)
    for _ in range(iters):
        gx, gy = grad(div(px, py) - f / theta)
        nrm = 1.0 + tau * np.sqrt(gx * gx + gy * gy)
        px = (px + tau * gx) / nrm
        py = (py + tau * gy) / nrm
    return f - theta * div(px, py)


def texture(img_u8, prm: TvL1Params):
    f = np.asarray(img_u8, np.float64) / 255.0
    return f - prm.alpha * rof(f, prm.theta_s, prm.tau_s, prm.iters_s)


def bilinear_clamped(img, x, y):
    """Bilinear samples of img at (x, y) arrays, coordinates clamped to the
    image (pixel centres at integers)."""
    H, W = img.shape
    x = np.clip(x, 0.0, W - 1.0)
    y = np.clip(y, 0.0, H - 1.0)
    x0 = np.floor(x).astype(np.int64)
    y0 = np.floor(y).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    a = x - x0
    b = y - y0
    return ((1 - a) * (1 - b) * img[y0, x0] + a * (1 - b) * img[y0, x1] +
            (1 - a) * b * img[y1, x0] + a * b * img[y1, x1])


def central_gradient(img):
    """(I(x+1) - I(x-1)) / 2 with clamped indices, both axes."""
    xp = np.concatenate([img[:, 1:], img[:, -1:]], axis=1)
    xm = np.concatenate([img[:, :1], img[:, :-1]], axis=1)
    yp = np.concatenate([img[1:, :], img[-1:, :]], axis=0)
    ym = np.concatenate([img[:1, :], img[:-1, :]], axis=0)
    return 0.5 * (xp - xm), 0.5 * (yp - ym)


def data_step(u1, u2, gx, gy, rho0, lam_theta):
    """v minimising |v - u|^2 / (2 theta) + lam |rho0 + g . v| pointwise:
    a step of lam*theta along -sign(rho) g where |rho(u)| is large, else the
    projection onto rho = 0; u itself where the gradient vanishes."""
    g2 = gx * gx + gy * gy
    rho = rho0 + gx * u1 + gy * u2
    t = lam_theta * g2
    s = np.zeros_like(u1)
    lo = rho < -t
    hi = rho > t
    mid = ~lo & ~hi & (g2 > 0)
    s[lo] = lam_theta
    s[hi] = -lam_theta
    s[mid] = -rho[mid] / g2[mid]
    return u1 + s * gx, u2 + s * gy


def tvl1_level(I0, I1, u1, u2, prm: TvL1Params, return_dual: bool = False):
    """Warps and iterations at one level from the initial flow (u1, u2)."""
    H, W = I0.shape
    xs, ys = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    Ix, Iy = central_gradient(I1)
    p = [np.zeros_like(I0) for _ in range(4)]       # p1x, p1y, p2x, p2y
    lt = prm.lam * prm.theta
    k = prm.tau / prm.theta
    shrink = 1.0 + prm.tau * prm.eps / prm.theta
    for _ in range(prm.warps):
        wx = xs + u1
        wy = ys + u2
        I1w = bilinear_clamped(I1, wx, wy)
        gx = bilinear_clamped(Ix, wx, wy)
        gy = bilinear_clamped(Iy, wx, wy)
        rho0 = I1w - gx * u1 - gy * u2 - I0
        for _ in range(prm.iters):
            v1, v2 = data_step(u1, u2, gx, gy, rho0, lt)
            u1 = v1 + prm.theta * div(p[0], p[1])
            u2 = v2 + prm.theta * div(p[2], p[3])
            for c, u in ((0, u1), (2, u2)):
                ax, ay = grad(u)
                qx = (p[c] + k * ax) / shrink
                qy = (p[c + 1] + k * ay) / shrink
                n = np.maximum(1.0, np.sqrt(qx * qx + qy * qy))
                p[c] = qx / n
                p[c + 1] = qy / n
    if return_dual:
        return u1, u2, p
    return u1, u2


def upsample_flow(u, W, H):
    """Flow of a finer level W x H from level-l flow u: 2 u(x / 2)."""
    xs, ys = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    return 2.0 * bilinear_clamped(u, 0.5 * xs, 0.5 * ys)


def tvl1_flow(pyr0: list, pyr1: list, prm: TvL1Params, perturb: float = 0.0):
    """Dense flow (u1, u2) at level 0 of two uint8 pyramids (lists of levels,
    at least prm.levels each).  perturb > 0 adds a fixed pattern of that
    amplitude to every texture: a probe of how far the result moves under
    input changes the size of float32 rounding (the conditioning of the
    problem, the yardstick for comparing a float32 run)."""
    L = prm.levels
    u1 = u2 = None
    for l in range(L - 1, -1, -1):
        I0 = texture(pyr0[l], prm)
        I1 = texture(pyr1[l], prm)
        H, W = I0.shape
        if perturb:
            ys, xs = np.mgrid[0:H, 0:W]
            pat = perturb * (((xs * 7 + ys * 13) % 17) - 8) / 8.0
            I0, I1 = I0 + pat, I1 - pat
        if u1 is None:
            u1 = np.zeros((H, W))
            u2 = np.zeros((H, W))
        else:
            u1 = upsample_flow(u1, W, H)
            u2 = upsample_flow(u2, W, H)
        u1, u2 = tvl1_level(I0, I1, u1, u2, prm)
    return u1, u2


def box_mean_flow(u1, u2, boxes):
    """Per box: mean of the flow over the pixels with integer centres inside
    the box (edges included, clipped to the image); the box moves by it.
    Returns (out_boxes (m,4), count (m,), mean (m,2)); no pixel -> unchanged."""
    H, W = u1.shape
    boxes = np.asarray(boxes, np.float64).reshape(-1, 4)
    out = boxes.copy()
    cnt = np.zeros(len(boxes), np.int64)
    mean = np.zeros((len(boxes), 2))
    for b, (x0, y0, x1, y1) in enumerate(boxes):
        xa, xb = max(0, int(np.ceil(x0))), min(W - 1, int(np.floor(x1)))
        ya, yb = max(0, int(np.ceil(y0))), min(H - 1, int(np.floor(y1)))
        if xa > xb or ya > yb:
            continue
        m1 = u1[ya:yb + 1, xa:xb + 1].mean()
        m2 = u2[ya:yb + 1, xa:xb + 1].mean()
        cnt[b] = (xb - xa + 1) * (yb - ya + 1)
        mean[b] = (m1, m2)
        out[b] += (m1, m2, m1, m2)
    return out, cnt, mean
