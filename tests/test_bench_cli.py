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
    sha = bench.cast_source_sha256()
    assert sha is not None and len(sha) == 64
    t = bench.traffic_bytes()
    rec = bench.K_CAST_TRAFFIC
    if rec is not None and sha == rec["source_sha256"]:
        assert t == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    else:
        assert t is None


def test_kernel_rates_are_algorithmic_flop_over_launch_time():
    sys.path.insert(0, ROOT)
    import bench
    # 2 launches of 1 ms each, 1e9 tests: 5e8 tests per launch x 16 FLOP / 1 ms = 8 TFLOP/s
    avg_ms, per_launch, tflops, gbps = bench.kernel_rates(2.0, 2, 1_000_000_000, 2_000_000_000)
    assert avg_ms == 1.0 and per_launch == 5e8
    assert abs(tflops - 8.0) < 1e-9 and abs(gbps - 1000.0) < 1e-9
