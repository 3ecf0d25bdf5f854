"""Host-side checks of the benchmark script (no GPU needed)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_traffic_table_covers_every_tuned_jacobi_shape():
    """The tuner's Jacobi candidates are tile heights 8..128 (x 256 columns)
    on 64..512 units with at most one wavefront per tile row; the headline's
    roofline looks its measured HBM traffic up by (tile height, units), so
    every candidate needs an entry, and each entry lies between the
    algorithmic bytes of a 4096^2 sweep and 1.1 times them."""
    alg = 4 * 4096 * 4096 + 4 * 4094 * 4094
    for th in (8, 16, 32, 64, 128):
        for units in (64, 128, 256, 512):
            if units > th * 64:
                continue
            t = bench.JACOBI_4096_TRAFFIC[(th, units)]
            assert alg <= t <= 1.1 * alg, (th, units, t)
