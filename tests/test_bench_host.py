"""Host checks of the benchmark script (no GPU): the one-GPU contract, and
that the committed HBM counter summary of the headline kernel was taken on
its current sources (otherwise the bench reports roofline.traffic as null)."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert p.returncode != 0
    assert "one GPU" in p.stderr


def test_headline_traffic_matches_current_sources():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        data = json.load(fh)
    for key in ("k_stage/sto10k/f32", "k_stage/sto10k/f64"):
        rec = data[key]
        assert rec["source_hash"] == bench.kernel_source_hash("k_stage"), key
        # HBM bytes within a few percent of the algorithmic N^2 b per launch
        elem = 4 if key.endswith("f32") else 8
        assert 1.0 <= rec["hbm_bytes_per_launch"] / (1e8 * elem) <= 1.05, key
