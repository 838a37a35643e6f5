"""bench.py contract pieces that run without a GPU: the refusal of more than
one GPU, and the algorithmic byte counts the roofline uses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus must be 1" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes():
    # read H (B U complex64) and y once, write z (complex64) and sigma2 (float32)
    assert bench.bytes_per_system(256, 16) == 256 * 16 * 8 + 256 * 8 + 16 * 8 + 16 * 4 == 35008
    assert bench.bytes_per_system(1024, 32) == 270720
    # several vectors: S receive vectors in, S estimates out, one sigma2 row
    assert bench.bytes_per_system_sym(256, 16, 14) == 256 * 16 * 8 + 14 * 256 * 8 + 14 * 16 * 8 + 16 * 4 == 63296
