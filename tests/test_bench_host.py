"""Host-side logic of bench.py (no GPU): the multi-GPU refusal, the metric
helpers and the committed counter summary it reads."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_flops_per_contribution():
    # alpha (11) + compositing (4) + K_code multiply-adds
    assert bench.flops_per_contribution(8) == 31
    assert bench.flops_per_contribution(0) == 15


def test_counter_summary_is_parsed_and_tied_to_the_source():
    h = bench.composite_source_hash()
    assert len(h) == 16
    path = os.path.join(ROOT, "profiles", "composite_scene_1M_200views_hbm_counters.md")
    txt = open(path).read()
    t = bench.measured_traffic()
    if f"source_sha256: {h}" in txt:
        assert t is not None and t > 0
    else:
        assert t is None
