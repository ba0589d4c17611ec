"""Host-side contract of bench.py (no GPU): one GPU only, the algorithmic
byte count of a stage launch, and the measured-traffic record that is only
reported for the kernel sources it was measured with."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_launch():
    # 2D N=4, 131072 triangles, FP32: 3.75 passes of K Np NF 4 bytes plus
    # 72 bytes of vertex coordinates and ids per triangle
    K, Np, NF = 131072, 15, 6
    b = bench.algorithmic_bytes_per_launch(K, Np, NF, 2, 4)
    assert b == 3.75 * K * Np * NF * 4 + K * (3 * 2 * 8 + 2 * 3 * 4)
    assert abs(b / 1e6 - 186.38) < 0.01
    # tetrahedra: 4 vertices x 3 coordinates x 8 bytes + 8 ids x 4 bytes
    assert bench.algorithmic_bytes_per_launch(1, 20, 10, 3, 4) == 3.75 * 200 * 4 + 4 * 3 * 8 + 2 * 4 * 4


def test_measured_traffic_follows_the_sources():
    K = bench.MEASURED_TRAFFIC["K"]
    saved = dict(bench.MEASURED_TRAFFIC)
    try:
        bench.MEASURED_TRAFFIC["sha256"] = bench.sources_digest()
        assert bench.measured_traffic(K) == bench.MEASURED_TRAFFIC["bytes_per_launch"]
        assert bench.measured_traffic(K + 16) is None
        bench.MEASURED_TRAFFIC["sha256"] = "0" * 64
        assert bench.measured_traffic(K) is None
    finally:
        bench.MEASURED_TRAFFIC.update(saved)
