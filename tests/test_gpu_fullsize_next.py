"""Parity at the full sizes of the walk-on-stars and implicit-boundary
workloads, in the launch configuration the benchmark times (FP32, all points
in one call).

* Thermal design (65,536-segment zero-flux slice, 16384 points on it with
  their walks starting on the wall, 256 walks): sampled per-point solutions
  against the oracle under the statistical parity rule; over all points,
  reverse mode equals the weighted forward mode of the same walks.
* Curve inflation (32 monopoles, the ~6,000 pixels inside the domain of a
  128 x 128 image, W = 4 with K = 4 nested walks): the squared-loss
  U-statistic gradient and loss equal their definition evaluated on the
  per-walk records of the same walks; sampled pixels against the oracle.
"""
import numpy as np
import pytest

import scenes
from helpers import parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def dwos():
    import paper_2405_12964_amd as m
    return m


def T(x, dev):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=dev)


def _se(v):
    return np.sqrt(np.maximum(np.asarray(v, float), 0))


def test_thermal_fullsize(dev, dwos, oracle_mod):
    sc = scenes.thermal_scene()
    X, seg = scenes.points_on_segments(sc.NV, sc.nsegs, 16384, 1)
    s = dwos.Solver.from_scene(sc, "fp32")
    s.set_start_segments(seg)
    Xt = T(X, dev)
    m, v = s.solve(Xt, 256, 11)
    idx = np.random.default_rng(5).choice(len(X), 8, replace=False)
    om, ov, _ = oracle_mod.Oracle(sc).solve(X[idx], 512, 12, start_seg=seg[idx])
    print(parity(m.cpu().numpy()[idx], _se(v.cpu().numpy()[idx]), om, _se(ov), abs_tol=1e-4,
                 name="thermal solve, sampled"))
    # forward mode at the sampled points (64 wire-shape parameters)
    ud_s, uv_s, _ = s.jvp(Xt, 256, 14)
    oud, ouv, _, _ = oracle_mod.Oracle(sc).jvp(X[idx], 256, 15, start_seg=seg[idx])
    print(parity(ud_s.cpu().numpy()[idx], _se(uv_s.cpu().numpy()[idx]), oud, _se(ouv), abs_tol=1e-4,
                 name="thermal jvp, sampled"))
    del ud_s, uv_s
    w = np.random.default_rng(6).normal(size=len(X))
    ud, _, _ = s.jvp(Xt, 16, 13, var=False)
    g, _ = s.grad(Xt, T(w, dev), 16, 13)
    ref = (T(w, dev)[:, None] * ud).sum(0)
    assert np.allclose(g.cpu().numpy(), ref.cpu().numpy(), rtol=1e-6, atol=1e-9 * float(ref.abs().max()))


def test_inflation_fullsize(dev, dwos, oracle_mod):
    side = 128
    g1 = -1.0 + (np.arange(side) + 0.5) * 2.0 / side
    Xall = np.stack(np.meshgrid(g1, g1), -1).reshape(-1, 2)
    sc = scenes.inflation_scene(32, seed=2).with_(K=4)
    s = dwos.Solver.from_scene(sc, "fp32")
    _, reg = s.implicit_band_grad(T(Xall, dev), T(np.zeros(len(Xall)), dev), 4.0 / side, want_mask=True)
    X = Xall[reg.cpu().numpy() == 2]
    assert len(X) > 4000
    Xt = T(X, dev)
    uref = np.random.default_rng(7).uniform(0.0, 0.4, len(X))
    W = B = 4
    L, g, um = s.grad_sqloss(Xt, T(uref, dev), W, B, 21)
    rec = s.walk_records(Xt, W, 21, mode=1, udot=True)
    u = rec["u"].cpu().numpy()
    ud = rec["udot"].cpu().numpy()
    S = u.sum(1, keepdims=True)
    omega = ((S - u) / (B * (B - 1)) - uref[:, None] / B) / (W // B)
    gref = np.einsum("pw,pwj->j", omega, ud)
    assert np.allclose(g.cpu().numpy(), gref, rtol=1e-9, atol=1e-12 * np.abs(gref).max())
    assert np.allclose(um.cpu().numpy(), u.mean(1), rtol=0, atol=1e-12)
    assert abs(float(L) - 0.5 * np.sum((u.mean(1) - uref) ** 2)) < 1e-9 * max(1.0, float(L))
    idx = np.random.default_rng(8).choice(len(X), 32, replace=False)
    m, v = s.solve(T(X[idx], dev), 4096, 22)
    om, ov, _ = oracle_mod.Oracle(sc).solve(X[idx], 4096, 23)
    print(parity(m.cpu().numpy(), _se(v.cpu().numpy()), om, _se(ov), name="inflation solve, sampled"))
