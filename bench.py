"""Benchmark of the MI355X pyramidal Lucas-Kanade tracking path.

One step = one frame pair of the 720x576 box scene (20 textured moving
rectangles, 8000 grid points, window 21x21, 4 levels, 30 iterations,
eps 0.01): build the new frame's pyramid, track every point, update every
box.  The previous frame's pyramid is resident (steady state), every input
is in HBM before the timed region, and each step is one HIP-graph replay.

Prints ONE JSON line with the throughput (tracked points/s), the roofline of
the dominant kernel (Lucas-Kanade, bound by FP32 vector ALU) and the CPU
oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tracked points/s (LK 21×21, 4 lvls) + p99 frame latency, served vs plain"
PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector, published (packed issue)
PEAK_FP32_UNPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 flop x 2.4 GHz, one FP32 op per lane
PEAK_HBM_GBS = 8000.0

# Algorithmic FP32 work of the tracker per point and level (the method's per-pixel formulation):
FLOP_TEMPLATE = 441 * 27     # 3 bilinear samples (7 flop) + 3 tensor FMAs (6 flop) per window pixel
FLOP_SCHARR = 22 * 22 * 20   # 2 fused Scharr responses (10 flop) per bilinear tap
FLOP_ITER = 441 * 12         # bilinear (7) + mismatch (1) + two FMAs (4) per window pixel


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    p.add_argument("--profile-only", action="store_true",
                   help="run only the timed GPU region (for rocprofv3)")
    p.add_argument("--profile-extra", action="store_true",
                   help="run only the Median-Flow step and the matching step (for rocprofv3)")
    p.add_argument("--copy-calib", action="store_true",
                   help="run a plain 256 MiB device copy (scale for the HBM byte counters)")
    p.add_argument("--no-batched", action="store_true", help="skip the 32-stream batched tick")
    p.add_argument("--no-served", action="store_true", help="skip the served-vs-plain run")
    p.add_argument("--no-video", action="store_true",
                   help="skip the one-stream video run with and without prefetch")
    p.add_argument("--no-dense", action="store_true",
                   help="skip the dense TV-L1 flow + mean-flow box prediction step")
    p.add_argument("--no-working", action="store_true",
                   help="skip the 1920x1080 full-resolution vs working-level comparison")
    p.add_argument("--no-match", action="store_true",
                   help="skip the matching/update step (IoU on the GPU, assignment on the host)")
    p.add_argument("--no-mf", action="store_true",
                   help="skip the Median-Flow step (forward-backward tracking, scaled boxes)")
    p.add_argument("--served-seconds", type=float, default=60.0,
                   help="length of the 64-stream arrival trace at 25 fps, served and plain")
    p.add_argument("--served-rates", default="1,2,4,6,8,12,16,24,32",
                   help="arrival-rate multipliers on 25 fps per stream for the saturation "
                        "sweep (comma list; stops once the served p99 passes 40 ms)")
    p.add_argument("--sweep-seconds", type=float, default=3.0,
                   help="trace length of each saturation-sweep rate")
    return p.parse_args()


def lk_kernel_flops(iters: np.ndarray, lam: np.ndarray) -> float:
    """Algorithmic flops of one tracking launch from its per-level diagnostics:
    a level counts its set-up when it was reached (lambda recorded) and
    FLOP_ITER per iteration it ran."""
    reached = (lam != 0.0)
    return float(reached.sum() * (FLOP_TEMPLATE + FLOP_SCHARR) + iters.astype(np.int64).sum() * FLOP_ITER)


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in ("ot_device.hpp", "ot_lk_dev.hpp", "ot_lk_sched.hpp", "ot_lk.hip", "ot_common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1910_06017_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def lk_kernel_name(win: int, margin: int) -> str:
    """The tracker instance a single-call launch of this window and margin runs."""
    m = margin or 4  # the library's default margin
    return f"k_lk_track<7,{win},{m}>" if win == 21 and m in (4, 6) else "k_lk_track<7>"


def traffic_from_profile(launch_pts: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "lk_sd_boxes_counters.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_sha") != kernel_sha() or d.get("points") != launch_pts:
        return None
    return d.get("hbm_bytes_per_launch")


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                          "(independent streams would be placed on GPUs whole, by HBM budget and load)"}))
        sys.exit(2)
    import torch
    from paper_1910_06017_amd import ops, synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    torch.cuda.init()
    dev = torch.device("cuda:0")
    if a.copy_calib:
        x = torch.empty(256 << 20, dtype=torch.uint8, device=dev).fill_(1)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel(), "copies": 3}))
        return
    wl = synth.sd_boxes_workload()
    L, WIN, ITERS, EPS = wl.levels, wl.win, wl.iters, wl.eps
    H, W = wl.frame0.shape
    f0 = torch.from_numpy(wl.frame0).to(dev)
    f1 = torch.from_numpy(wl.frame1).to(dev)
    pts = torch.from_numpy(wl.pts).to(dev)
    boxes = torch.from_numpy(wl.boxes).to(dev)
    bid = torch.from_numpy(wl.box_id).to(dev)
    n, m = wl.n, wl.boxes.shape[0]
    prev = ops.pyramid_build(f0, L)
    ws1 = ops.alloc_workspace(W, H, L)
    from paper_1910_06017_amd import batch
    # the step builds the next pyramid, which is the next step's template
    # pyramid: materialized gradients would have to be built every step, so
    # the step takes the fastest schedule with gradients computed in the tracker
    MARGIN = batch.default_schedule("single_" + batch.bucket_key(
        [type("J", (), {"n": n, "levels": L})()]), grads=False).get("margin", 0)
    nxt = torch.empty((n, 2), dtype=torch.float32, device=dev)
    st = torch.empty(n, dtype=torch.uint8, device=dev)
    err = torch.empty(n, dtype=torch.float32, device=dev)
    ob = torch.empty((m, 4), dtype=torch.float32, device=dev)
    oc = torch.empty(m, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    def step():
        Q = ops.pyramid_build(f1, L, ws=ws1)
        ops.lk_track(prev, Q, pts, win=WIN, levels=L, iters=ITERS, eps=EPS, margin=MARGIN,
                     out=(nxt, st, err))
        ops.box_update(boxes, bid, pts, nxt, st, out=(ob, oc))

    nxt_pyr = ops.pyramid_build(f1, L, ws=ws1)

    def lk_only():
        ops.lk_track(prev, nxt_pyr, pts, win=WIN, levels=L, iters=ITERS, eps=EPS, margin=MARGIN,
                     out=(nxt, st, err))

    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        step()
        lk_only()
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()
    g_step, g_lk = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_step, stream=cs):
        step()
    with torch.cuda.graph(g_lk, stream=cs):
        lk_only()
    torch.cuda.synchronize()

    for _ in range(a.warmup):
        g_step.replay()
    torch.cuda.synchronize()
    # ---- timed region: K whole steps
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(cs)
    with torch.cuda.stream(cs):
        for _ in range(a.steps):
            g_step.replay()
    t1.record(cs)
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / a.steps
    if a.profile_only:
        print(json.dumps({"ms_per_step": ms_step}))
        return
    if a.profile_extra:
        print(json.dumps({"median_flow": bench_median_flow(a, ops, wl, prev, f1, ws1, pts, boxes, bid,
                                                           WIN, L, ITERS, EPS, MARGIN, cs,
                                                           scenes=False),
                          "matching": bench_matching(ops, wl, ob, cs)}))
        return

    # ---- per-step latency distribution (events around each replay)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(min(a.steps, 200))]
    with torch.cuda.stream(cs):
        for e0, e1 in evs:
            e0.record(cs)
            g_step.replay()
            e1.record(cs)
    torch.cuda.synchronize()
    lat = np.array([e0.elapsed_time(e1) for e0, e1 in evs])

    # ---- dominant kernel: Lucas-Kanade launches alone, events on its stream
    reps = max(20, a.steps)
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(cs):
        for _ in range(5):
            g_lk.replay()
        k0.record(cs)
        for _ in range(reps):
            g_lk.replay()
        k1.record(cs)
    torch.cuda.synchronize()
    lk_ms = k0.elapsed_time(k1) / reps

    # ---- cold step: both frames' pyramids built (no resident template pyramid)
    ws0 = ops.alloc_workspace(W, H, L)

    def cold_step():
        P0 = ops.pyramid_build(f0, L, ws=ws0)
        Q = ops.pyramid_build(f1, L, ws=ws1)
        ops.lk_track(P0, Q, pts, win=WIN, levels=L, iters=ITERS, eps=EPS, margin=MARGIN,
                     out=(nxt, st, err))
        ops.box_update(boxes, bid, pts, nxt, st, out=(ob, oc))

    with torch.cuda.stream(cs):
        cold_step()
    torch.cuda.synchronize()
    g_cold = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_cold, stream=cs):
        cold_step()
    cold_ms = _graph_ms(torch, g_cold, cs, max(20, a.steps))
    _, _, _, it, lam = ops.lk_track(prev, nxt_pyr, pts, win=WIN, levels=L, iters=ITERS, eps=EPS,
                                    want_diag=True)
    torch.cuda.synchronize()
    flops = lk_kernel_flops(it.cpu().numpy(), lam.cpu().numpy())
    achieved = flops / (lk_ms * 1e-3) / 1e12
    ok_frac = float(st.float().mean().item())

    out = {
        "metric": METRIC,
        "value": n / (ms_step * 1e-3),
        "unit": "tracked points/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "cold": {"ms_per_step": cold_ms, "tracked_points_per_s": n / (cold_ms * 1e-3),
                 "step": "both frames' pyramids + LK + per-box median, one HIP graph replay"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "720x576 frame pair, 20 moving textured boxes, 8000 grid points, "
                               "LK window 21x21, 4 levels, 30 iterations, eps 0.01; step = "
                               "next-frame pyramid + LK + per-box median, one HIP graph replay",
                   "points_per_step": n, "boxes": m, "levels": L, "win": WIN,
                   "lds_margin": MARGIN},
        "frame_latency_ms": {"p50": float(np.percentile(lat, 50)),
                             "p99": float(np.percentile(lat, 99)), "path": "plain"},
        "ok_fraction": ok_frac,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": traffic_from_profile(n),
                     "kernel": lk_kernel_name(WIN, MARGIN), "kernel_ms": lk_ms,
                     "flop_per_launch": flops,
                     "frac_of_unpacked_fp32": achieved / PEAK_FP32_UNPACKED_TFLOPS},
    }
    if not a.no_mf:
        out["median_flow"] = bench_median_flow(a, ops, wl, prev, f1, ws1, pts, boxes, bid,
                                               WIN, L, ITERS, EPS, MARGIN, cs)
    if not a.no_match:
        out["matching"] = bench_matching(ops, wl, ob, cs)
    if not a.no_working:
        out["working_level"] = bench_working_level(ops, cs)
    if not a.no_dense:
        out["dense_tvl1"] = bench_dense(ops, wl, f0, f1, boxes, cs)
    if not a.no_batched:
        out["batched"] = bench_batched(a)
    if not a.no_video:
        out["video_prefetch"] = bench_video(a)
    if not a.no_video and not a.no_dense:
        out["dense_video"] = bench_dense_video(a)
    if not a.no_served:
        out["served_vs_plain"] = bench_served(a)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_seconds)
    print(json.dumps(out))


def _graph_ms(torch, g, cs, reps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(cs):
        for _ in range(3):
            g.replay()
        e0.record(cs)
        for _ in range(reps):
            g.replay()
        e1.record(cs)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_median_flow(a, ops, wl, prev, f1, ws1, pts, boxes, bid, WIN, L, ITERS, EPS, MARGIN, cs,
                      scenes=True):
    """The Median-Flow step on the same frame pair: next pyramid, forward and
    backward tracking, the forward-backward gate (1 px) and the scaled box
    update, one graph replay; the gate and the scaled update are also timed
    alone, and (scenes) the scaled update on a few large boxes."""
    import torch
    dev = pts.device
    n, m = pts.shape[0], boxes.shape[0]
    nxt = torch.empty((n, 2), dtype=torch.float32, device=dev)
    back = torch.empty((n, 2), dtype=torch.float32, device=dev)
    sf = torch.empty(n, dtype=torch.uint8, device=dev)
    sb = torch.empty(n, dtype=torch.uint8, device=dev)
    st = torch.empty(n, dtype=torch.uint8, device=dev)
    fe = torch.empty(n, dtype=torch.float32, device=dev)
    ob = torch.empty((m, 4), dtype=torch.float32, device=dev)
    oc = torch.empty(m, dtype=torch.int32, device=dev)
    osc = torch.empty(m, dtype=torch.float32, device=dev)
    wsc = ops.box_scaled_workspace(m, dev)
    kw = dict(win=WIN, levels=L, iters=ITERS, eps=EPS, margin=MARGIN)
    Q = ops.pyramid_build(f1, L, ws=ws1)

    def step():
        ops.pyramid_build(f1, L, ws=ws1)
        ops.lk_track_fb(prev, Q, pts, out=(nxt, sf, None, back, sb), fb_max=1.0,
                        gate_out=(st, fe), **kw)
        ops.box_update_scaled(boxes, bid, pts, nxt, st, out=(ob, oc, osc), ws=wsc)

    def step_two():
        ops.pyramid_build(f1, L, ws=ws1)
        ops.lk_track(prev, Q, pts, out=(nxt, sf, None), **kw)
        ops.lk_track(Q, prev, nxt, out=(back, sb, None), **kw)
        ops.fb_gate(pts, back, sf, sb, 1.0, out=(st, fe))
        ops.box_update_scaled(boxes, bid, pts, nxt, st, out=(ob, oc, osc), ws=wsc)

    def gate():
        ops.fb_gate(pts, back, sf, sb, 1.0, out=(st, fe))

    def scaled():
        ops.box_update_scaled(boxes, bid, pts, nxt, st, out=(ob, oc, osc), ws=wsc)

    # the step is one replay; each kernel alone is KREP launches per replay so
    # that the graph's own launch cost is amortised
    KREP = 10
    graphs = []
    for fn, k in ((step, 1), (gate, KREP), (scaled, KREP), (step_two, 1)):
        with torch.cuda.stream(cs):
            fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=cs):
            for _ in range(k):
                fn()
        graphs.append(g)
    torch.cuda.synchronize()
    reps = max(20, a.steps)
    ms = _graph_ms(torch, graphs[0], cs, reps)
    gate_ms = _graph_ms(torch, graphs[1], cs, reps) / KREP
    sc_ms = _graph_ms(torch, graphs[2], cs, reps) / KREP
    ms_two = _graph_ms(torch, graphs[3], cs, reps)
    c = oc.cpu().numpy().astype(np.int64)
    pairs = int((c * (c - 1) // 2).sum())
    gate_bytes = n * (8 + 8 + 1 + 1 + 1 + 4)
    return {"ms_per_step": ms, "value": n / (ms * 1e-3), "unit": "tracked points/s",
            "step": "next pyramid + LK forward and backward with the FB gate (1 px) in one "
                    "launch + scaled box update",
            "ms_per_step_two_launches": ms_two,
            "kept_fraction": float(st.float().mean().item()),
            "fb_gate_us": gate_ms * 1e3,
            "fb_gate_hbm_frac": gate_bytes / (gate_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "box_scaled_us": sc_ms * 1e3, "box_pairs": pairs,
            "box_pairs_per_s": pairs / (sc_ms * 1e-3),
            "box_scaled_scenes": bench_scaled_scenes(ops, dev, cs, reps, KREP) if scenes else None}


def bench_scaled_scenes(ops, dev, cs, reps, krep):
    """The scaled box update alone on seeded point sets of few large boxes
    (similarity motion, 10 % outliers, 5 % lost points): 20 boxes of 400
    points, 16 of 1000, 4 of 5000; krep launches per graph replay."""
    import torch
    from paper_1910_06017_amd import synth
    out = {}
    for name, counts, seed in (("20x400", [400] * 20, 1), ("16x1000", [1000] * 16, 2),
                               ("4x5000", [5000] * 4, 3)):
        arrs = [torch.from_numpy(np.ascontiguousarray(x)).to(dev)
                for x in synth.similarity_box_points(seed, counts)]
        mm = arrs[0].shape[0]
        o = (torch.empty((mm, 4), dtype=torch.float32, device=dev),
             torch.empty(mm, dtype=torch.int32, device=dev),
             torch.empty(mm, dtype=torch.float32, device=dev))
        w2 = ops.box_scaled_workspace(mm, dev)

        def fn():
            ops.box_update_scaled(*arrs, out=o, ws=w2)

        with torch.cuda.stream(cs):
            fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=cs):
            for _ in range(krep):
                fn()
        torch.cuda.synchronize()
        us = _graph_ms(torch, g, cs, reps) / krep * 1e3
        c = o[1].cpu().numpy().astype(np.int64)
        pairs = int((c * (c - 1) // 2).sum())
        out[name] = {"us": us, "pairs": pairs, "pairs_per_s": pairs / (us * 1e-6)}
    return out


def bench_dense(ops, wl, f0, f1, boxes, cs):
    """The dense variant on the same frame pair: TV-L1 flow with the default
    parameters (both frames' structure-texture split, 5 levels, 5 warps x 30
    iterations) and the mean-flow box prediction, one graph replay; with the
    structure-texture split on a second stream ahead of the flow (the
    default), and with everything on one stream."""
    import torch
    p = ops.tvl1_params()
    H, W = wl.frame0.shape
    P = ops.pyramid_build(f0, p.levels)
    Q = ops.pyramid_build(f1, p.levels)
    ws = torch.empty(int(ops.lib().ot_tvl1_bytes(W, H)), dtype=torch.uint8, device=f0.device)
    aux = torch.cuda.Stream(f0.device)  # default priority
    res, flows = {}, {}
    for name, a in (("two_streams", aux), ("one_stream", None)):
        flow = torch.empty((H, W, 2), dtype=torch.float32, device=f0.device)
        ob = torch.empty_like(boxes)
        oc = torch.empty(boxes.shape[0], dtype=torch.int32, device=f0.device)

        def step():
            ops.tvl1_flow(P, Q, p, ws=ws, out=flow, stream=cs, aux_stream=a)
            ops.box_mean_flow(flow, boxes, out=(ob, oc), stream=cs)

        with torch.cuda.stream(cs):
            step()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=cs):
            step()
        res[name] = _graph_ms(torch, g, cs, 10)
        flows[name] = flow.clone()
    ms = res["two_streams"]
    px = W * H
    # one iteration kernel at level 0: read u 8 B, p 16 B, data 16 B; write u 8 B, p 16 B
    it_bytes = px * 64
    # Algorithmic bytes of the step's passes over every level, counted per
    # iteration as if each read its inputs from and wrote its outputs to HBM:
    # TV-L1 iteration 64 B/pixel; structure dual iteration per frame: p in and
    # out 16 B + the uint8 level 1 B; warp: I0, I1 4 B each, gradient 8 B,
    # flow 8 B, data out 16 B = 40 B; texture per frame: level 1 B, p 8 B,
    # texture out 4 B; gradient: texture 4 B in, 8 B out.
    alg = 0
    for l in range(p.levels):
        n = P.desc.w[l] * P.desc.h[l]
        alg += n * (p.warps * p.iters * 64 + p.iters_s * 2 * 17 + p.warps * 40 + 2 * 13 + 12)
    achieved = alg / (ms * 1e-3) / 1e9
    return {"ms_per_step": ms, "frames_per_s": 1e3 / ms, "pixels_per_s": px / (ms * 1e-3),
            "ms_per_step_one_stream": res["one_stream"],
            "roofline": {"bound": "hbm", "kernel": "whole dense step (all levels' passes)",
                         "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                         "frac": achieved / 8000.0, "traffic": None,
                         "algorithmic_bytes_per_step": alg},
            "identical": bool(torch.equal(flows["two_streams"], flows["one_stream"])),
            "levels": p.levels, "warps": p.warps, "iters": p.iters, "iters_s": p.iters_s,
            "iter_bytes_level0": it_bytes,
            "step": "TV-L1 flow (structure-texture of both frames, all levels, on a second "
                    "stream ahead of the flow) + box mean"}


def bench_working_level(ops, cs):
    """The 1920x1080 box scene (14,400 points, window 21) tracked at full
    resolution (5 levels) and at its working level (level 1, 4 levels):
    next-frame pyramid + tracking per graph replay."""
    import torch
    from paper_1910_06017_amd import synth
    w = synth.hd_boxes_workload()
    dev = torch.device("cuda:0")
    f0 = torch.from_numpy(w.frame0).to(dev)
    f1 = torch.from_numpy(w.frame1).to(dev)
    pts = torch.from_numpy(w.pts).to(dev)
    n = pts.shape[0]
    base = ops.working_level(w.W, w.H)
    res = {"workload": "1920x1080, 16 boxes, 14400 points, window 21, 30 iterations",
           "level": base}
    for name, b, L in (("full_resolution", 0, 5), ("working_level", base, 5 - base)):
        prev = ops.pyramid_build(f0, b + L)
        ws = ops.alloc_workspace(w.W, w.H, b + L)
        nxt = torch.empty((n, 2), dtype=torch.float32, device=dev)
        st = torch.empty(n, dtype=torch.uint8, device=dev)

        def step():
            Q = ops.pyramid_build(f1, b + L, ws=ws)
            ops.lk_track(prev, Q, pts, levels=L, base_level=b, out=(nxt, st, None))

        with torch.cuda.stream(cs):
            step()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=cs):
            step()
        ms = _graph_ms(torch, g, cs, 50)
        res[name] = {"levels": L, "base_level": b, "ms_per_step": ms,
                     "tracked_points_per_s": n / (ms * 1e-3),
                     "ok_fraction": float(st.float().mean().item())}
    return res


def bench_matching(ops, wl, pred, cs):
    """The matching and update phases after one step of the box scene:
    scores of the 20 predicted boxes against synthetic detections (true
    next boxes, 1 px jitter, 10 % missed, 2 new) on the GPU, then the
    optimal assignment and the update on the host.  Also a 30 x 32 case
    (the largest box count of the mixed streams)."""
    import torch
    from paper_1910_06017_amd import synth
    res = {}
    rng = np.random.default_rng(7)
    cases = [("sd_boxes", pred, synth.detections(wl.boxes_next, rng, wl.W, wl.H))]
    S30 = rng.uniform(0, 1800, (30, 2))
    S30 = np.concatenate([S30, S30 + rng.uniform(40, 200, (30, 2))], axis=1).astype(np.float32)
    cases.append(("30x32", torch.from_numpy(S30).to(pred.device),
                  synth.detections(S30, rng, 1920, 1080, miss=0.0, extra=2)))
    KREP = 10
    for name, S, det in cases:
        D = torch.from_numpy(det).to(S.device)
        iou = torch.empty((S.shape[0], D.shape[0]), dtype=torch.float32, device=S.device)
        with torch.cuda.stream(cs):
            ops.iou_matrix(S, D, out=iou)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=cs):
            for _ in range(KREP):
                ops.iou_matrix(S, D, out=iou)
        iou_us = _graph_ms(torch, g, cs, 50) / KREP * 1e3
        # one full step as a caller runs it: scores, copy back, host phases
        m, k = S.shape[0], D.shape[0]
        Sh = S.cpu().numpy()
        B = np.zeros((m + k, 4), np.float32)
        I = np.zeros(m + k, np.int32)
        L = np.zeros(m + k, np.uint8)
        # the scores come back through pinned memory on the compute stream
        ih_pin = torch.empty((m, k), dtype=torch.float32, pin_memory=True)
        ts = []
        for _ in range(50):
            t0 = time.perf_counter()
            with torch.cuda.stream(cs):
                ops.iou_matrix(S, D, out=iou)
                ih_pin.copy_(iou, non_blocking=True)
            cs.synchronize()
            ih = ih_pin.numpy()
            s2d, d2s, score = ops.assign(ih, 0.3)
            B[:m] = Sh
            I[:m] = np.arange(m)
            L[:m] = 0
            mo, _ = ops.track_update(B, I, L, m, det, s2d, d2s, m)
            ts.append(time.perf_counter() - t0)
        t_as = []
        for _ in range(50):
            t0 = time.perf_counter()
            ops.assign(ih, 0.3)
            t_as.append(time.perf_counter() - t0)
        res[name] = {"objects": m, "detections": k, "matched": int((s2d >= 0).sum()),
                     "iou_kernel_us": iou_us, "assign_host_us": float(np.median(t_as)) * 1e6,
                     "step_us_median": float(np.median(ts)) * 1e6,
                     "step": "IoU on the GPU + copy to host + assignment + update"}
    return res


def bench_batched(a):
    """32 independent streams (mixed 720x576 / 1280x720 / 1920x1080, 4-30 boxes,
    500-20000 points each) in one batched tick, replayed as a HIP graph."""
    import torch
    from paper_1910_06017_amd import batch, ops, synth

    ws = synth.batched_streams()
    jobs = batch.jobs_from_workloads(ws, "cuda:0")
    npts = sum(w.n for w in ws)
    sched = batch.default_schedule(batch.bucket_key(jobs))
    # the graph's capacities fitted to the tick (jobs, points, boxes, pyramid
    # tiles): a graph sized past them dispatches idle workgroups every replay
    cfg = batch.fit_capacities(batch.BatchConfig(max_jobs=32, max_points=npts, max_boxes=2048,
                                                 max_tiles=1 << 15, max_levels=5, **sched), jobs)
    runner = batch.BatchRunner(cfg, tables=1)
    runner.pack(jobs, table=0)
    g = runner.capture(0)
    for _ in range(5):
        g.replay()
    torch.cuda.synchronize()
    reps = 30
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = float(np.mean([j.status.float().mean().item() for j in jobs if j.n]))
    # the tracking stage alone (batched tracker + box median) on the packed
    # table, events on its stream; its algorithmic flops from every point's
    # per-level iteration counts (the per-stream call gives the same bits)
    import ctypes as C
    cs = torch.cuda.Stream()
    h = int(cs.cuda_stream)
    run = lambda st: ops.check(ops.lib().ot_batch_run_stages(
        int(runner.host[0].data_ptr()), int(runner.dev.data_ptr()), runner.table_bytes,
        C.byref(runner.ccfg), st, h), "ot_batch_run_stages")
    with torch.cuda.stream(cs):
        run(1)
        for _ in range(3):
            run(2)
        k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        k0.record(cs)
        for _ in range(reps):
            run(2)
        k1.record(cs)
    torch.cuda.synchronize()
    trk_ms = k0.elapsed_time(k1) / reps
    flops = 0.0
    for j, Qb in zip(jobs, runner.next_pyrs):
        if j.n:
            _, _, _, it, lam = ops.lk_track(j.prev, Qb, j.pts, win=cfg.win, levels=j.levels,
                                            iters=cfg.iters, eps=cfg.eps, want_diag=True)
            flops += lk_kernel_flops(it.cpu().numpy(), lam.cpu().numpy())
    achieved = flops / (trk_ms * 1e-3) / 1e12
    return {"streams": len(ws), "points_per_tick": npts, "ms_per_tick": ms,
            "tracked_points_per_s": npts / (ms * 1e-3), "schedule": sched,
            "capacities": {"jobs": cfg.max_jobs, "points": cfg.max_points,
                           "boxes": cfg.max_boxes, "tiles": cfg.max_tiles}, "ok_fraction": ok,
            "tracking_stage_ms": trk_ms,
            "roofline": {"bound": "alu", "kernel": "k_lk_batch<7,21,4,1,1> + k_batch_box",
                         "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_FP32_TFLOPS,
                         "frac_of_unpacked_fp32": achieved / PEAK_FP32_UNPACKED_TFLOPS,
                         "flop_per_tick": flops}}


def bench_served(a):
    """64 streams with Poisson arrivals at 25 fps each, served with continuous
    batching (two ticks in flight: the next tick's uploads and pyramids
    overlap the current tracking) and, on the same trace, plain per-stream
    calls: the full-length trace at the configured rate, then short traces at
    rising rates until the served p99 passes one frame interval (40 ms)."""
    from paper_1910_06017_amd import serve, synth

    streams = synth.served_streams(nframes=10)
    specs = [serve.StreamSpec(s.sid, s.W, s.H, s.levels, sum(s.pts_per_box), len(s.pts_per_box))
             for s in streams]
    pinned = [[_pin(f) for f in s.frames] for s in streams]
    seeds = {}

    def frame_fn(sid, k, t):
        s = streams[sid]
        reseed = None
        if k % 10 == 0:
            key = (sid, k % len(s.frames))
            if key not in seeds:
                seeds[key] = s.seed_points(k, np.random.default_rng(sid * 7919 + k))
            reseed = seeds[key]
        return serve.Frame(sid, k, t, pinned[sid][k % len(s.frames)], reseed)

    pts_of = {s.sid: sum(s.pts_per_box) for s in streams}
    executors = {"served": (True, serve.GpuExecutor(max_jobs=64, max_points=1 << 21)),
                 "served_blocking": (True, serve.GpuExecutor(max_jobs=64, max_points=1 << 21,
                                                             depth=1)),
                 "plain": (False, serve.PlainExecutor())}
    # warm every path (allocation, first launches) on a short trace
    warm = serve.make_trace(len(streams), 0.2, 25.0, seed=1)
    for name, (batched, ex) in executors.items():
        serve.run_trace(warm, frame_fn, specs, serve.Scheduler(1 << 40, 64, 1 << 21), ex,
                        batched=batched)
        for sid in list(ex.slots):
            ex.evict(sid)

    def run(name, seconds, rate):
        batched, ex = executors[name]
        trace = serve.make_trace(len(streams), seconds, 25.0, seed=505, rate_scale=rate)
        sch = serve.Scheduler(budget=1 << 40, max_jobs=64, max_points=1 << 21)
        ex.ticks = 0
        t0 = time.perf_counter()
        res = serve.run_trace(trace, frame_fn, specs, sch, ex, batched=batched,
                              max_wall=seconds * 3)
        wall = time.perf_counter() - t0
        st = serve.latency_stats(res)
        st["completed"] = len(res)
        st["all_completed"] = len(res) == len(trace)
        st["tracked_points_per_s"] = sum(pts_of[r.sid] for r in res if r.k > 0) / max(wall, 1e-9)
        st["ticks"] = ex.ticks
        st["frames_per_tick"] = len(res) / max(1, ex.ticks)
        for sid in list(ex.slots):
            ex.evict(sid)
        offered = sum(pts_of[s] for _, s, _ in trace) / seconds
        return len(trace), offered, st

    full = {"rate": 1.0, "fps_per_stream": 25.0, "trace_s": a.served_seconds}
    for name in ("served", "plain"):
        nfr, offered, st = run(name, a.served_seconds, 1.0)
        full["frames"], full["offered_points_per_s"] = nfr, offered
        full[name] = st
        print(f"served_vs_plain: {name} {a.served_seconds:.0f} s at 1x: p50 "
              f"{st['p50_ms']:.3f} p99 {st['p99_ms']:.3f} ms", file=sys.stderr, flush=True)
    runs, live = [], {"served", "served_blocking", "plain"}
    for rate in [float(r) for r in a.served_rates.split(",")]:
        rec = {"rate": rate, "fps_per_stream": 25.0 * rate, "trace_s": a.sweep_seconds}
        for name in ("served", "served_blocking", "plain"):
            if name not in live:
                continue
            nfr, offered, st = run(name, a.sweep_seconds, rate)
            rec["frames"], rec["offered_points_per_s"] = nfr, offered
            rec[name] = st
            if not st["all_completed"] or st["p99_ms"] > 40.0:
                live.discard(name)          # saturated: higher rates only queue more
        runs.append(rec)
        print(f"served_vs_plain: sweep rate {rate:g} done, still under 40 ms: {sorted(live)}",
              file=sys.stderr, flush=True)
        if "served" not in live:
            break
    # the largest offered load each path serves with p99 <= 40 ms (one 25 fps
    # frame interval) and every frame completed
    sat = {}
    for name in ("served", "served_blocking", "plain"):
        ok = [r["offered_points_per_s"] for r in runs
              if name in r and r[name]["all_completed"] and r[name]["p99_ms"] <= 40.0]
        bad = [r["offered_points_per_s"] for r in runs
               if name in r and not (r[name]["all_completed"] and r[name]["p99_ms"] <= 40.0)]
        sat[name] = {"max_ok": max(ok) if ok else None, "first_over": min(bad) if bad else None}
    return {"streams": len(streams), "full_trace": full, "sweep": runs,
            "saturation_points_per_s": sat}


def bench_dense_video(a):
    """One 720x576 stream tracked densely frame by frame (TV-L1 defaults, the
    mean flow inside each of 20 boxes), 30 frames from pinned host memory
    (a 12-frame cycle, re-seeded every 10th): each frame's upload, pyramid
    and structure-texture split computed once, on the tracking stream or
    prefetched on a second one."""
    import torch
    from paper_1910_06017_amd import ops, synth, video

    W, H, nbox = 720, 576, 20
    s = synth.served_streams(seed=607, nstreams=1, nframes=12, npts_range=(8000, 8000),
                             nbox_range=(nbox, nbox), resolutions=((W, H),))[0]
    cyc = [_pin(f) for f in s.frames]
    frames = [cyc[k % len(cyc)] for k in range(30)]
    seeds = {k: s.seed_points(k, np.random.default_rng(k))[2] for k in range(0, 30, 10)}
    p = ops.tvl1_params()
    rec = {"frames": len(frames), "boxes": nbox, "levels": p.levels, "warps": p.warps,
           "iters": p.iters, "iters_s": p.iters_s}
    results = {}
    for key, pf in (("one_stream", False), ("prefetch", True)):
        trk = video.DenseVideoTracker(W, H, p, m_max=nbox, prefetch=pf)
        trk.track(frames[:6], seeds)            # warm-up
        torch.cuda.synchronize()
        best = None
        for _ in range(2):
            t0 = time.perf_counter()
            res = trk.track(frames, seeds)
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        results[key] = res
        rec[key] = {"ms_per_frame": 1e3 * best / (len(frames) - 1),
                    "frames_per_s": (len(frames) - 1) / best}
    rec["identical"] = all(np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
                           for x, y in zip(results["one_stream"], results["prefetch"]))
    rec["speedup_prefetch"] = rec["one_stream"]["ms_per_frame"] / rec["prefetch"]["ms_per_frame"]
    return rec


def bench_video(a):
    """One stream tracked frame by frame from pinned host frames, at the
    working level of its resolution: everything on one stream; the next
    frame's upload and pyramid prefetched on a second stream (Sec. V-B); and
    prefetched with the points tracked longest-first by their iteration counts
    in the previous pair; and prefetched with each frame's Scharr planes built
    with its pyramid.  SD (720x576, level 0) and the 2K (2560x1280, level
    1) and 4K (4096x2048, level 2) sizes of the paper's runtime experiment,
    each a 12-frame cycle played 5 times (60 frames, re-seeded every 10th)."""
    import torch
    from paper_1910_06017_amd import ops, synth, video

    out = {}
    for (W, H), npts, nbox in (((720, 576), 8000, 20), ((2560, 1280), 8000, 12),
                               ((4096, 2048), 12000, 16)):
        s = synth.served_streams(seed=606, nstreams=1, nframes=12, npts_range=(npts, npts),
                                 nbox_range=(nbox, nbox), resolutions=((W, H),))[0]
        cyc = [_pin(f) for f in s.frames]
        frames = [cyc[k % len(cyc)] for k in range(60)]
        seeds = {k: s.seed_points(k, np.random.default_rng(k)) for k in range(0, 60, 10)}
        base = ops.working_level(W, H)
        rec = {"frames": len(frames), "points": npts, "boxes": nbox, "working_level": base,
               "levels": 4}
        results = {}
        for key, pf, order, grads in (("one_stream", False, False, False),
                                      ("prefetch", True, False, False),
                                      ("prefetch_order", True, True, False),
                                      ("prefetch_grads", True, False, True)):
            trk = video.VideoTracker(W, H, levels=4, base_level=base, n_max=npts, m_max=nbox,
                                     prefetch=pf, order=order, grads=grads)
            trk.track(frames[:12], seeds)           # warm-up
            torch.cuda.synchronize()
            best = None
            for _ in range(3):
                t0 = time.perf_counter()
                res = trk.track(frames, seeds)
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            results[key] = res
            rec[key] = {"ms_per_frame": 1e3 * best / (len(frames) - 1),
                        "frames_per_s": (len(frames) - 1) / best,
                        "tracked_points_per_s": npts * (len(frames) - 1) / best}
        rec["identical"] = all(np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
                               for k in ("prefetch", "prefetch_order", "prefetch_grads")
                               for x, y in zip(results["one_stream"], results[k]))
        base_ms = rec["one_stream"]["ms_per_frame"]
        rec["speedup_prefetch"] = base_ms / rec["prefetch"]["ms_per_frame"]
        rec["speedup_prefetch_order"] = base_ms / rec["prefetch_order"]["ms_per_frame"]
        rec["speedup_prefetch_grads"] = base_ms / rec["prefetch_grads"]["ms_per_frame"]
        out[f"{W}x{H}"] = rec
    return out


def _pin(frame):
    import torch
    t = torch.empty(frame.shape, dtype=torch.uint8, pin_memory=True)
    t.copy_(torch.from_numpy(frame))
    return t


def cpu_model() -> str:
    """The host CPU's model name (lscpu / /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _oracle_steps(wl, seconds: float, nthreads: int, pts=None):
    """Whole oracle steps (next-frame pyramid, tracking, box update) on one
    frame pair until `seconds` have passed (at least one); returns (steps,
    points per step, seconds)."""
    import oracle

    pts = wl.pts if pts is None else pts
    sel = None if pts is wl.pts else slice(0, len(pts))
    prev = oracle.pyramid(wl.frame0, wl.levels)
    steps, t0 = 0, time.perf_counter()
    while True:
        nxt = oracle.pyramid(wl.frame1, wl.levels)
        r = oracle.lk_track_pyr(prev, nxt, pts, wl.win, wl.levels, wl.iters,
                                float(np.float32(wl.eps)), nthreads=nthreads)
        if sel is None:
            oracle.box_update(wl.boxes, wl.box_id, wl.pts, r.next_pts, r.status)
        steps += 1
        dt = time.perf_counter() - t0
        if dt >= seconds:
            return steps, len(pts), dt


def cpu_baseline(wl, seconds: float):
    """The FP64 oracle on the host cores: whole steps (next-frame pyramid,
    tracking, box update) on the 720x576 box scene, repeated for ~`seconds`,
    with every host thread.  `detail` adds the shifted-texture, box-scene and
    1080p pairs and one 32-stream tick, each with all threads and with one
    (bounded samples: ~2 s per entry, the tick on every 8th point of each
    stream at one thread)."""
    import oracle
    from paper_1910_06017_amd import synth

    oracle.build(force=not os.path.exists(oracle.LIB_PATH))
    threads = oracle.max_threads()
    steps, npts, dt = _oracle_steps(wl, seconds, 0)
    out = {"value": steps * npts / dt, "unit": "tracked points/s", "cores": threads,
           "kind": "oracle", "cpu": cpu_model(), "host_threads": os.cpu_count(),
           "sample": f"{steps} whole steps of the same 720x576 box-scene frame pair "
                     f"({npts} points), {dt:.1f} s, FP64, OpenMP over points"}
    detail = {}
    cases = {"720x576 shifted texture, 1024 points, 3 levels": synth.sd_shift_workload(),
             "720x576 boxes, 8000 points, 4 levels": wl,
             "1920x1080 boxes, 14400 points, 5 levels": synth.hd_boxes_workload()}
    for name, w in cases.items():
        rec = {}
        for nt, key in ((threads, "all_threads"), (1, "one_thread")):
            s_, n_, d_ = _oracle_steps(w, 2.0, nt)
            rec[key] = {"points_per_s": s_ * n_ / d_, "ms_per_step": 1e3 * d_ / s_,
                        "threads": nt, "steps": s_}
        detail[name] = rec
    ws = synth.batched_streams()
    rec = {}
    for nt, key, stride in ((threads, "all_threads", 1), (1, "one_thread", 8)):
        t0, npts = time.perf_counter(), 0
        for w in ws:
            p = w.pts[::stride]
            _oracle_steps(w, 0.0, nt, pts=p if stride > 1 else None)
            npts += len(p)
        d_ = time.perf_counter() - t0
        rec[key] = {"points_per_s": npts / d_, "threads": nt, "points": npts,
                    "seconds": d_,
                    "sample": "every point" if stride == 1 else f"every {stride}th point"}
    detail["32-stream tick (mixed 720x576/1280x720/1920x1080), 169567 points"] = rec
    out["detail"] = detail
    return out


if __name__ == "__main__":
    main()
