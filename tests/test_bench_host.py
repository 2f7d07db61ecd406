"""Host logic of the benchmark (no GPU): the committed HBM counter summaries
are used only for the kernel sources and nested-walk count they were taken
on; the fixed-RMSE rule recovers a known noise level."""
import os
import re

import numpy as np
import pytest

import bench


@pytest.mark.parametrize("workload,kernel", [("c2", "walk_kernel<float,2,1,true,false>"),
                                             ("c3", "walk_kernel<float,3,1,false,false>")])
def test_traffic_figure_matches_sources_and_workload(workload, kernel):
    path = bench.TRAFFIC_FILES[workload]
    if not os.path.exists(path):
        assert bench.measured_traffic(kernel, 1, workload) is None
        return
    with open(path) as f:
        text = f.read()
    kv = dict(re.findall(r"^# (\w+): (\S+)$", text, re.M))
    K = int(kv["nested_walks_per_terminal"])
    t = bench.measured_traffic(kernel, K, workload)
    if kv["sources_sha256"] != bench.sources_sha256():
        assert t is None      # counters of other kernel sources are not reported
        return
    assert t is not None and t > 0
    assert bench.measured_traffic(kernel, K + 1, workload) is None


def test_traffic_needs_the_summary(monkeypatch, tmp_path):
    monkeypatch.setitem(bench.TRAFFIC_FILES, "c2", os.path.join(tmp_path, "missing.txt"))
    assert bench.measured_traffic("walk_kernel<float,2,1,true,false>", 8, "c2") is None


class _FakeGrad:
    """Stands in for a solver: gradients g* + noise of variance s2 * 64 / W,
    a known unbiased estimator (the rule's arithmetic only, no walks)."""

    def __init__(self, gstar, s2, seed=0):
        self.gstar, self.s2 = np.asarray(gstar, float), s2
        self.rng = np.random.default_rng(seed)

    def grad(self, X, w, W, seed, u_mean=False):
        import torch
        sd = np.sqrt(self.s2 * 64.0 / W)
        return torch.tensor(self.gstar + sd * self.rng.normal(size=self.gstar.size)), None


def test_fixed_rmse_rule_recovers_known_noise(monkeypatch):
    torch = pytest.importorskip("torch")
    monkeypatch.setattr(torch.cuda, "synchronize", lambda: None)
    gstar = np.random.default_rng(1).normal(size=4096)
    # relative RMSE at W = 256: sqrt(s2 * 64 / 256) / 1 = 0.5 -> W* = 256 * 25 = 6400
    fake = _FakeGrad(gstar, 1.0)
    r = bench.grad_rmse_rate(fake, None, None, W_probe=256, reps=12, W_time_max=512)
    rms = float(np.sqrt(np.mean(gstar ** 2)))
    assert abs(r["rel_rmse_at_probe"] - 0.5 / rms) < 0.05 / rms
    assert abs(r["walks_per_point"] / (6400 / rms ** 2) - 1) < 0.1
    assert r["extrapolated"] and r["timed_walks_per_point"] == 512
