"""The offset-point gradient estimator of the normal derivative
(eq. (dudn_mc_estimate), the paper's ablation; dwos_problem.dudn = 1) on the
GPU against the FP64 oracle, through the C ABI.

* Walk for walk: the FP64 walk kernel reproduces every oracle walk (u,
  step count, terminal primitive, nested estimate, udot) within 1e-9 in 2D
  (mapped data, K = 2) and 3D (harmonic data).
* FP32: the mapped disk's du/dR closed form, statistical parity with the
  oracle, reverse mode equal to the weighted forward mode.
* The RMSE of both estimators on the same derivative (printed).
* Error paths: screened or sourced problems, the control variate, a
  reflecting or an implicit boundary.
"""
import numpy as np
import pytest

import scenes
from helpers import check_vs_exact, parity

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


def T(x, dev, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device=dev)


def _se(v):
    return np.sqrt(np.maximum(np.asarray(v, float), 0))


def _harmonic3(sc):
    return sc.with_(bc=[dict(kind="restricted", c=0.0, b=np.zeros(3), A=np.diag([1.0, -1.0, 0.0]))])


def _wfw(dev, dwos, oracle_mod, sc, X, W, seed):
    s = dwos.Solver.from_scene(sc, "fp64")
    o = oracle_mod.Oracle(sc)
    g = s.walk_records(T(X, dev), W, seed, mode=1, udot=True)
    r = o.walk_records(X, W, seed, mode=1)
    assert np.allclose(g["u"].cpu().numpy(), r["u"], rtol=0, atol=1e-9)
    assert np.array_equal(g["steps"].cpu().numpy(), r["steps"])
    assert np.array_equal(g["prim"].cpu().numpy(), r["prim"])
    go = g["uoff"].cpu().numpy()
    assert np.allclose(go, r["uoff"], rtol=0, atol=1e-9), np.abs(go - r["uoff"]).max()
    gd = g["udot"].cpu().numpy()
    scale = max(1.0, float(np.abs(r["udot"]).max()))
    assert np.allclose(gd, r["udot"], rtol=0, atol=1e-9 * scale), np.abs(gd - r["udot"]).max()


def test_walk_for_walk_2d_and_3d(dev, dwos, oracle_mod):
    sc = scenes.c1_polygon(128, mapped=True, eps=1e-4, delta=1e-2, K=2).with_(dudn=1)
    _wfw(dev, dwos, oracle_mod, sc, scenes.points_in_disk(12, 0.85, 81), 16, 82)
    sc = _harmonic3(scenes.sphere_scene(8, eps=1e-4, delta=1e-2)).with_(dudn=1, K=3)
    _wfw(dev, dwos, oracle_mod, sc, scenes.points_in_ball(8, 0.0, 0.8, 83), 8, 84)


def test_fp32_closed_form_parity_and_reverse_mode(dev, dwos, oracle_mod):
    sc = scenes.c1_polygon(128, mapped=True, eps=1e-4, delta=1e-3).with_(dudn=1, K=2)
    X = scenes.points_in_disk(128, 0.8, 85)
    s = dwos.Solver.from_scene(sc, "fp32")
    ud, uv, _ = s.jvp(T(X, dev), 16384, 86)
    check_vs_exact(ud.cpu().numpy()[:, 0], _se(uv.cpu().numpy()[:, 0]), -2 * (X[:, 0] ** 2 - X[:, 1] ** 2),
                   5e-3, "gradient-estimator dudR fp32")
    Xs = X[:48]
    ud, uv, _ = s.jvp(T(Xs, dev), 1024, 87)
    oud, ouv, _, _ = oracle_mod.Oracle(sc).jvp(Xs, 1024, 88)
    print(parity(ud.cpu().numpy()[:, 0], _se(uv.cpu().numpy()[:, 0]), oud[:, 0], _se(ouv[:, 0]),
                 name="gradient-estimator jvp fp32"))
    w = np.random.default_rng(89).normal(size=len(X))
    ud, _, _ = s.jvp(T(X, dev), 256, 90, var=False)
    g, _ = s.grad(T(X, dev), T(w, dev), 256, 90)
    ref = (T(w, dev)[:, None] * ud).sum(0)
    assert np.allclose(g.cpu().numpy(), ref.cpu().numpy(), rtol=1e-6, atol=1e-9 * float(ref.abs().max()))


def test_estimator_rmse(dev, dwos):
    """RMSE of du/dR on the mapped disk (exact -2(x^2 - y^2)) for both
    estimators at equal walk counts, over 1024 points and 8 repetitions."""
    X = scenes.points_in_disk(1024, 0.8, 91)
    exact = -2 * (X[:, 0] ** 2 - X[:, 1] ** 2)
    Xt = T(X, dev)
    out = {}
    for dudn in (0, 1):
        s = dwos.Solver.from_scene(scenes.c1_polygon(256, mapped=True, eps=1e-3, delta=1e-2).with_(dudn=dudn),
                                   "fp32")
        errs = []
        for rep in range(8):
            ud, _, _ = s.jvp(Xt, 64, 100 + rep, var=False)
            errs.append(ud.cpu().numpy()[:, 0] - exact)
        out[dudn] = float(np.sqrt(np.mean(np.square(errs))))
    print(f"du/dR RMSE at 64 walks per point: backward difference {out[0]:.4f}, "
          f"gradient estimator {out[1]:.4f} (ratio {out[0] / out[1]:.3f})")
    assert np.isfinite(out[0]) and np.isfinite(out[1])


def test_gradient_estimator_error_paths(dev, dwos):
    from paper_2405_12964_amd.capi import DwosError, DWOS_EINVAL, DWOS_ESTATE
    from paper_2405_12964_amd.solver import make_problem
    s = dwos.Solver(2, "fp32")
    for kw in (dict(sigma=1.0), dict(src_c0=1.0), dict(dudn=2)):
        args = dict(sigma=0.0, src_c0=0.0, dudn=1, dim=2)
        args.update(kw)
        with pytest.raises(DwosError) as e:
            s.set_problem(make_problem(**args))
        assert e.value.code == DWOS_EINVAL
    X = T(scenes.points_in_disk(4, 0.5, 92), dev)
    # a reflecting boundary
    ls = scenes.lshape_scene().with_(dudn=1)
    sl = dwos.Solver.from_scene(ls, "fp32")
    with pytest.raises(DwosError) as e:
        sl.walk_records(T(scenes.points_in_lshape(4, 1), dev), 4, 1, mode=1)
    assert e.value.code == DWOS_ESTATE and "gradient normal-derivative" in str(e.value)
    sl.solve(T(scenes.points_in_lshape(4, 1), dev), 4, 1)      # forward walks are unaffected
    # an implicit boundary
    sm = dwos.Solver.from_scene(scenes.monopole_scene([[0.5, 0.0, 0.0]], g=(0.0, None, None)).with_(dudn=1),
                                "fp32")
    with pytest.raises(DwosError) as e:
        sm.jvp(X, 4, 1)
    assert e.value.code == DWOS_ESTATE and "gradient normal-derivative" in str(e.value)
    # the control variate
    sc = scenes.c1_polygon(64, eps=1e-3, delta=1e-2).with_(dudn=1)
    sd = dwos.Solver.from_scene(sc, "fp32")
    from paper_2405_12964_amd import cv as cvmod
    B = np.random.default_rng(93).normal(size=(4, 2))
    th = np.random.default_rng(94).normal(size=cvmod.theta_size()) * 0.01
    net = dwos.Network(2, B, th)
    sd.attach_cv(net, 1.0)
    with pytest.raises(DwosError) as e:
        sd.jvp(X, 4, 1)
    assert e.value.code == DWOS_ESTATE and "gradient normal-derivative" in str(e.value)
