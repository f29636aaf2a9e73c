"""bench.py host-side contract (no GPU): one GPU only, and the traffic record
is tied to the ray-test kernel's source."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_is_reported_only_for_the_profiled_kernel_source():
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.raster_source_sha256()
    assert sha is not None and len(sha) == 64
    t = bench.traffic_bytes()
    if sha == bench.K_TEST_TRAFFIC["source_sha256"]:
        assert t == bench.K_TEST_TRAFFIC["fetch_bytes_per_launch"] + bench.K_TEST_TRAFFIC["write_bytes_per_launch"]
    else:
        assert t is None
