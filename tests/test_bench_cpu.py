"""Host logic of the benchmark (no GPU): the multi-GPU refusal, the
algorithmic flop count of a tracking launch (the per-unit figures of the
measurement plan: 11.9 k template and 9.7 k Scharr flops per reached level,
5.3 k per iteration), and the rule that HBM traffic is reported only from
counters taken on the current tracker sources."""
import json
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_gpus_above_one_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_flop_count_of_a_launch():
    assert bench.FLOP_TEMPLATE == 441 * 27 == 11907
    assert bench.FLOP_SCHARR == 22 * 22 * 20 == 9680
    assert bench.FLOP_ITER == 441 * 12 == 5292
    # three points, two levels: a level counts its set-up when the tracker
    # reached it (recorded a lambda) and every iteration it ran
    iters = np.array([[3, 0], [30, 5], [0, 0]], dtype=np.uint8)
    lam = np.array([[1.5, 0.0], [2.0, 3.0], [0.0, 0.0]], dtype=np.float32)
    want = 3 * (11907 + 9680) + (3 + 30 + 5) * 5292
    assert bench.lk_kernel_flops(iters, lam) == want


def test_traffic_reported_only_for_matching_sources(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    path = tmp_path / "profiles" / "lk_sd_boxes_counters.json"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sha", lambda: "abc")
    assert bench.traffic_from_profile(8000) is None            # no counters
    path.write_text(json.dumps({"kernel_sha": "abc", "points": 8000,
                                "hbm_bytes_per_launch": 123.5}))
    assert bench.traffic_from_profile(8000) == 123.5
    assert bench.traffic_from_profile(7999) is None            # another launch size
    path.write_text(json.dumps({"kernel_sha": "old", "points": 8000,
                                "hbm_bytes_per_launch": 123.5}))
    assert bench.traffic_from_profile(8000) is None            # sources changed since


def test_committed_counters_match_the_tracker_sources():
    """The committed counter summary was taken on the tracker as it stands
    (else the benchmark would report no traffic)."""
    d = json.load(open(os.path.join(ROOT, "profiles", "lk_sd_boxes_counters.json")))
    assert d["kernel_sha"] == bench.kernel_sha()
    assert d["points"] == 8000 and d["hbm_bytes_per_launch"] > 0
