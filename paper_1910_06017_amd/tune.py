"""Autotune the batched tick's tracking schedule on representative ticks.

Runs `batch.Autotuner` on the 32-stream mixed tick (~170k points) and on a
small 4-stream tick over `batch.schedule_space()` (LDS margin x waves per
workgroup x points per wave, or a persistent grid), times the LDS margin and
fused vs materialized Scharr of the single-call tracker on the 720x576 and
1080p box scenes, and writes the winners (per shape bucket) to
`tune_cache.json` next to this file (or to the path given), which
`batch.default_schedule` reads.

    python -m paper_1910_06017_amd.tune [out.json]
"""
import json
import os
import sys

from . import batch, synth


def tune_single(cache: dict, reps: int = 30):
    """LDS margin of the single-call tracker, with Scharr computed in the
    kernel or read from planes materialized with the template pyramid, on
    the 720x576 and 1080p box scenes."""
    import torch

    from . import ops

    for w in (synth.sd_boxes_workload(), synth.hd_boxes_workload()):
        dev = torch.device("cuda:0")
        f0 = torch.from_numpy(w.frame0).to(dev)
        Ps = {g: ops.pyramid_build(f0, w.levels, grads=g) for g in (False, True)}
        Q = ops.pyramid_build(torch.from_numpy(w.frame1).to(dev), w.levels)
        pts = torch.from_numpy(w.pts).to(dev)
        out = (torch.empty((w.n, 2), device=dev), torch.empty(w.n, dtype=torch.uint8, device=dev),
               torch.empty(w.n, device=dev))
        res = []
        for g in (False, True):
            for m in (2, 3, 4, 6, 8):
                P = Ps[g]
                f = lambda: ops.lk_track(P, Q, pts, win=w.win, levels=w.levels, iters=w.iters,
                                         eps=w.eps, margin=m, out=out)
                for _ in range(3):
                    f()
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    f()
                e1.record()
                torch.cuda.synchronize()
                res.append((e0.elapsed_time(e1) / reps, m, g))
        res.sort(key=lambda r: r[0])
        key = f"single_{single_key(w.n, w.levels)}"
        cache[key] = {"schedule": {"margin": res[0][1], "grads": res[0][2]}, "ms": res[0][0],
                      "all": [{"ms": ms, "margin": m, "grads": g} for ms, m, g in res]}
        print(key, json.dumps(cache[key]["schedule"]), f"{res[0][0]:.3f} ms", flush=True)


def single_key(n: int, levels: int) -> str:
    return batch.bucket_key([type("J", (), {"n": n, "levels": levels})()])


def main(out=None):
    out = out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
    tuner = batch.Autotuner(path=out)
    for ws in (synth.batched_streams(), synth.batched_streams(seed=405, nstreams=4)):
        jobs = batch.jobs_from_workloads(ws)
        npts = sum(w.n for w in ws)
        base = batch.BatchConfig(max_jobs=len(ws), max_points=npts, max_boxes=2048,
                                 max_tiles=1 << 15, max_levels=5)
        rec = tuner.tune(jobs, base, reps=10, warmup=3)
        print(batch.bucket_key(jobs), json.dumps(rec["schedule"]), f"{rec['ms']:.3f} ms",
              flush=True)
        for r in rec["all"]:
            print("   ", json.dumps(r), flush=True)
    tune_single(tuner.cache)
    with open(out, "w") as f:
        json.dump(tuner.cache, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else None)
