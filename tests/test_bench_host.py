"""Host-side check of the benchmark's bookkeeping (no GPU): the committed
HBM-traffic summary belongs to the vmult kernel sources as they are (bench.py
reports `roofline.traffic` only when the hash of those sources matches the one
the counters were taken with), and the measured traffic exceeds the
algorithmic bytes of the same vmult."""
import json

import bench


def test_traffic_summary_matches_kernel_sources():
    with open(bench.TRAFFIC_FILE) as fh:
        tr = json.load(fh)
    assert tr["kernel_hash"] == bench.kernel_hash()
    w = tr["workloads"]["sneddon_1024x1024_L3_Q2"]
    # 1024^2 + 3 local levels, Q2: 6 844 629 nodes, 1 709 236 leaf cells
    assert w["bytes_per_launch"] > bench.algorithmic_bytes(6844629, 1709236, 2)
