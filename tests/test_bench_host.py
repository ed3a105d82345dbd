"""Host-side check of the benchmark's bookkeeping (no GPU): bench.py reports
`roofline.traffic` from the committed HBM-traffic summary only while the
vmult kernel sources hash to the value the counters were taken with (null
otherwise), and a current summary's traffic exceeds the algorithmic bytes of
the same vmult."""
import json

import bench


def test_traffic_is_reported_only_for_the_profiled_kernel_sources(tmp_path):
    with open(bench.TRAFFIC_FILE) as fh:
        tr = json.load(fh)
    name = "sneddon_1024x1024_L3_Q2"
    if tr["kernel_hash"] == bench.kernel_hash():
        w = tr["workloads"][name]
        # 1024^2 + 3 local levels, Q2: 6 844 629 nodes, 1 709 236 leaf cells
        assert w["bytes_per_launch"] > bench.algorithmic_bytes(6844629, 1709236, 2)
        assert bench.load_traffic(name) == w["bytes_per_launch"]
    else:
        assert bench.load_traffic(name) is None
    # a summary taken with other kernel sources is never used
    stale = dict(tr, kernel_hash="0" * 16)
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(stale))
    assert bench.load_traffic(name, str(f)) is None
    assert bench.load_traffic("no_such_workload") is None
