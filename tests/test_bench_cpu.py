"""bench.py's host-side pieces: the algorithmic byte counts it divides by
(the per-pixel figures of the workloads: state read and written once,
inputs and output once), the traffic record lookup, and the refusal of
more than one GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_per_pixel():
    # d = 8: 60 state floats read and written (480 B), colour + 7 features +
    # variance + motion in, 3 floats out
    assert bench.algorithmic_bytes_per_pixel(8, 4) == 480 + (3 + 7) * 4 + 4 + 8 + 12 == 544
    assert bench.algorithmic_bytes_per_pixel(8, 2) == 524
    assert bench.algorithmic_bytes_per_pixel(10, 2) == 2 * 85 * 4 + (3 + 9) * 2 + 4 + 8 + 12 == 728
    assert bench.algorithmic_bytes_per_pixel(8, 4, motion=False) == 536
    # paper mode: 25 state floats, colour and motion in, output
    assert bench.algorithmic_bytes_per_pixel_paper(4) == 2 * 25 * 4 + 12 + 8 + 12 == 232
    # blend: beta (3d floats), predictor source, guide, output
    assert bench.blend_bytes_per_pixel(8, 4) == 96 + 28 + 12 + 12 == 148
    assert bench.blend_bytes_per_pixel(10, 2) == 120 + 18 + 24 == 162
    assert bench.blend_bytes_per_pixel(4, 4, paper=True) == 48 + 12 + 24 == 84


def test_traffic_record_only_for_the_current_kernels():
    rec = bench.load_traffic("c2")
    path = os.path.join(ROOT, "profiles", "traffic_c2.json")
    with open(path) as f:
        stored = json.load(f)
    if stored.get("kernel_source_sha256_16") == bench.kernel_source_hash():
        assert rec == stored["hbm_bytes_per_launch"]
    else:
        assert rec is None
    assert bench.load_traffic("no-such-workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
