"""The benchmark's command-line contract on the host (no GPU): more than one
GPU is refused with a message and a non-zero exit, and the source hash that
keys the committed HBM-traffic table covers the step kernel's sources."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_traffic_table_is_keyed_by_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.src_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    # a key that does not match yields no traffic figure rather than a stale one
    assert bench.traffic_from_profiles(["no_such_kernel"]) is None
