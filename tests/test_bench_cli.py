"""The benchmark's command line on the CPU: more than one GPU is refused with
a message before any device work, and the algorithmic byte counts it prices
the rooflines with are the documented per-pixel and per-node sums."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import bench
    # grid pass: 123 planes read and written, I_s, two normal targets, three warped samples
    assert bench.BYTES_PER_PX_ITER == 123 * 8 + 4 + 8 + 12 == 1008
    # quadtree: 366 B per pixel and 1230 B per node
    assert 4 * bench.TREE_PIXEL_FLOATS == 366 and 4 * bench.TREE_NODE_FLOATS == 1230
