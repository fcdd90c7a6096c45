"""Autotune the batched tick's tracking schedule on representative ticks.

Runs `batch.Autotuner` on the 32-stream mixed tick (~170k points) and on a
small 4-stream tick, and writes the winners (per shape bucket) to
`tune_cache.json` next to this file (or to the path given), which
`batch.default_schedule` reads.

    python -m paper_1910_06017_amd.tune [out.json]
"""
import json
import os
import sys

from . import batch, synth


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


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else None)
