"""Host logic of the benchmark (no GPU): the committed HBM counter summary
is used only for the kernel sources and nested-walk count it was taken on."""
import os
import re

import bench


def test_traffic_figure_matches_sources_and_workload():
    with open(bench.TRAFFIC_FILE) as f:
        text = f.read()
    kv = dict(re.findall(r"^# (\w+): (\S+)$", text, re.M))
    K = int(kv["nested_walks_per_terminal"])
    t = bench.measured_traffic("walk_kernel<float,2,1,true>", K)
    if kv["sources_sha256"] != bench.sources_sha256():
        assert t is None      # counters of other kernel sources are not reported
        return
    assert t is not None and t > 0
    assert bench.measured_traffic("walk_kernel<float,2,1,true>", K + 1) is None


def test_traffic_needs_the_summary(monkeypatch, tmp_path):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", os.path.join(tmp_path, "missing.txt"))
    assert bench.measured_traffic("walk_kernel<float,2,1,true>", 8) is None
