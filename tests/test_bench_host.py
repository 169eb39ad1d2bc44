"""Host-side logic of bench.py (no GPU): the multi-GPU refusal, the byte
model behind the roofline and the committed counter summary it reads."""
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


def test_byte_model_of_the_uplift():
    """Per view: Gaussians 44 B, region map 4 B per pixel, code table 8 B per
    slot, 8 B per code slot per distinct (Gaussian, region) pair; per step
    the accumulator is zeroed and read once (4 N M each) and N x K written."""
    assert bench.uplift_view_bytes(10, 4, 3, 2, 8, 0) == 440 + 48 + 128
    assert bench.uplift_view_bytes(0, 0, 0, 0, 8, 5) == 320
    assert bench.uplift_step_bytes(10, 64, 4, 1000) == 1000 + 2 * 4 * 10 * 64 + 8 * 10 * 4
    # the 1M-Gaussian scene at U_v = 0.8 M: about 98.6 MB per view
    per_view = bench.uplift_view_bytes(1_000_000, 1008, 756, 120, 8, 800_000)
    assert 97e6 < per_view < 100e6


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
