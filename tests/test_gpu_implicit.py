"""Walks on an implicit boundary (harmonic monopoles, Sec. 7.4) on the GPU
against the FP64 oracle, through the C ABI.

* Walk-for-walk: the FP64 instantiation of the implicit-boundary kernel
  reproduces every oracle walk (u, step count, terminal flag, nested mean,
  the 3n-vector udot) within 1e-9: one monopole (Poisson, screened with
  roulette, harmonic data) and a 16-monopole inflation blob.
* Reductions: forward mode, reverse mode and the squared-loss U-statistic
  equal the oracle's at FP64 on the same seeds, also with more monopoles
  than a block has threads and walk counts that leave a ragged tile.
* The band term of the shape derivative equals the oracle's (FP64 exactly,
  FP32 away from the band's edges).
* FP32: against the oracle on independent seeds and against the disk's
  closed forms.
* Error paths of the entry points.
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


def _h(mono, c, x):
    return c + sum(m[0] / np.hypot(x[..., 0] - m[1], x[..., 1] - m[2]) for m in mono)


def _disk_points(n, seed, p, rmax):
    rng = np.random.default_rng(seed)
    r = rmax * np.sqrt(rng.random(n))
    t = 2 * np.pi * rng.random(n)
    return np.stack([p[0] + r * np.cos(t), p[1] + r * np.sin(t)], 1), r


def _inside(mono, c, n, seed, lo=-0.8, hi=0.8, hmin=0.05):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(lo, hi, (40 * n, 2))
    pts = pts[_h(mono, c, pts) > hmin]
    assert len(pts) >= n
    return pts[:n]


# ------------------------------------------------------------ walk for walk --

def _wfw(dev, dwos, oracle_mod, sc, X, W, seed, modes=(0, 1)):
    s = dwos.Solver.from_scene(sc, "fp64")
    o = oracle_mod.Oracle(sc)
    Xt = T(X, dev)
    for mode in modes:
        g = s.walk_records(Xt, W, seed, mode=mode, udot=(mode == 1))
        r = o.walk_records(X, W, seed, mode=mode)
        gu = g["u"].cpu().numpy()
        assert np.allclose(gu, r["u"], rtol=0, atol=1e-9), (mode, np.abs(gu - r["u"]).max())
        assert np.array_equal(g["steps"].cpu().numpy(), r["steps"]), mode
        if mode == 1:
            assert np.array_equal(g["prim"].cpu().numpy(), r["prim"])
            assert np.allclose(g["uoff"].cpu().numpy(), r["uoff"], rtol=0, atol=1e-9)
            gd = g["udot"].cpu().numpy()
            scale = max(1.0, float(np.abs(r["udot"]).max()))
            assert np.allclose(gd, r["udot"], rtol=0, atol=1e-9 * scale), np.abs(gd - r["udot"]).max()


def test_walk_for_walk_one_monopole(dev, dwos, oracle_mod):
    p, a, c = (0.1, -0.2), 0.5, -1.0
    X, _ = _disk_points(12, 1, p, 0.45)
    _wfw(dev, dwos, oracle_mod, scenes.monopole_scene([[a, *p]], c=c, src_c0=4.0, eps=1e-3, delta=1e-2, K=2),
         X, 16, 31)
    sc = scenes.monopole_scene([[a, *p]], c=c, sigma=9.0, g=(1.0, [0.3, -0.2], None), eps=1e-3, delta=1e-2)
    _wfw(dev, dwos, oracle_mod, sc, X, 16, 32)
    sc = scenes.monopole_scene([[a, *p]], c=c, g=(0.0, None, [[1.0, 0.0], [0.0, -1.0]]), eps=1e-3, delta=1e-2)
    _wfw(dev, dwos, oracle_mod, sc, X, 16, 33)


def test_walk_for_walk_inflation_blob(dev, dwos, oracle_mod):
    sc = scenes.inflation_scene(16, seed=3)
    X = _inside(sc.mono, sc.mono_c, 16, 4)
    _wfw(dev, dwos, oracle_mod, sc, X, 8, 34)


# --------------------------------------------------------------- reductions --

def _big_scene(n, seed):
    """n small monopoles on a ring (n > 256 takes the one-group path of the
    gradient reduction)."""
    rng = np.random.default_rng(seed)
    t = 2 * np.pi * np.arange(n) / n
    mono = np.stack([rng.uniform(0.5, 1.5, n) * 0.6 / n, 0.5 * np.cos(t), 0.5 * np.sin(t)], 1)
    return scenes.monopole_scene(mono, c=-1.0, src_c0=4.0, eps=1e-3, delta=1e-2)


@pytest.mark.parametrize("which", ["blob", "ring300"])
def test_grad_jvp_sqloss_match_oracle_fp64(dev, dwos, oracle_mod, which):
    if which == "blob":
        sc = scenes.inflation_scene(16, seed=5)
        X = _inside(sc.mono, sc.mono_c, 37, 6)
    else:
        sc = _big_scene(300, 7)
        X = _inside(sc.mono, sc.mono_c, 37, 8, hmin=0.02)
    W, B = 6, 3                      # 222 walks: one ragged tile
    s = dwos.Solver.from_scene(sc, "fp64")
    o = oracle_mod.Oracle(sc)
    Xt = T(X, dev)
    rng = np.random.default_rng(9)
    w = rng.normal(size=len(X))
    uref = rng.uniform(0.0, 0.3, len(X))
    ud, uv, um = s.jvp(Xt, W, 41)
    oud, ouv, oum, _ = o.jvp(X, W, 41)
    sc_ = max(1.0, np.abs(oud).max())
    assert np.allclose(ud.cpu().numpy(), oud, rtol=0, atol=1e-9 * sc_)
    assert np.allclose(uv.cpu().numpy(), ouv, rtol=1e-6, atol=1e-12 * sc_ ** 2)
    assert np.allclose(um.cpu().numpy(), oum, rtol=0, atol=1e-9)
    g, gm = s.grad(Xt, T(w, dev), W, 42)
    og, ogm, _ = o.grad(X, w, W, 42)
    assert np.allclose(g.cpu().numpy(), og, rtol=0, atol=1e-9 * max(1.0, np.abs(og).max()))
    assert np.allclose(gm.cpu().numpy(), ogm, rtol=0, atol=1e-9)
    L, g2, m2 = s.grad_sqloss(Xt, T(uref, dev), W, B, 43)
    oL, og2, om2, _ = o.grad_sqloss(X, uref, W, B, 43)
    assert abs(float(L) - oL) < 1e-9 * max(1.0, abs(oL))
    assert np.allclose(g2.cpu().numpy(), og2, rtol=0, atol=1e-9 * max(1.0, np.abs(og2).max()))


def test_band_grad_matches_oracle(dev, dwos, oracle_mod):
    sc = scenes.inflation_scene(16, seed=11)
    g1 = np.linspace(-0.9, 0.9, 301)
    X = np.stack(np.meshgrid(g1, g1), -1).reshape(-1, 2)
    rng = np.random.default_rng(12)
    coef = rng.uniform(0.5, 1.5, len(X))
    eps_band = 0.02
    og, om = oracle_mod.Oracle(sc).band_grad(X, coef, eps_band)
    assert (om == 1).sum() > 100 and (om == 2).sum() > 100 and (om == 0).sum() > 100
    s = dwos.Solver.from_scene(sc, "fp64")
    g0 = rng.normal(size=sc.N)
    g, m = s.implicit_band_grad(T(X, dev), T(coef, dev), eps_band, grad=T(g0, dev), want_mask=True)
    assert np.array_equal(m.cpu().numpy(), om)
    assert np.allclose(g.cpu().numpy() - g0, og, rtol=1e-11, atol=1e-11 * np.abs(og).max())
    # FP32: drop the points whose band decision is within rounding of an edge
    h = _h(sc.mono, sc.mono_c, X)
    ok = np.abs(h) > 1e-4
    gr = np.zeros_like(X)
    for m_ in sc.mono:
        d = X - m_[1:]
        gr -= m_[0] * d / np.linalg.norm(d, axis=1)[:, None] ** 3
    ok &= np.abs(h - eps_band * np.linalg.norm(gr, axis=1)) > 1e-4
    og2, om2 = oracle_mod.Oracle(sc).band_grad(X[ok], coef[ok], eps_band)
    g32, m32 = dwos.Solver.from_scene(sc, "fp32").implicit_band_grad(T(X[ok], dev), T(coef[ok], dev), eps_band,
                                                                      want_mask=True)
    assert np.array_equal(m32.cpu().numpy(), om2)
    assert np.allclose(g32.cpu().numpy(), og2, rtol=1e-4, atol=1e-5 * np.abs(og2).max())


# ----------------------------------------------------------------- FP32 -----

def test_fp32_parity_and_closed_forms(dev, dwos, oracle_mod):
    sc = scenes.inflation_scene(16, seed=13)
    X = _inside(sc.mono, sc.mono_c, 48, 14)
    s = dwos.Solver.from_scene(sc, "fp32")
    m, v = s.solve(T(X, dev), 2048, 51)
    om, ov, _ = oracle_mod.Oracle(sc).solve(X, 2048, 52)
    print(parity(m.cpu().numpy(), _se(v.cpu().numpy()), om, _se(ov), name="inflation u fp32"))
    ud, uv, _ = s.jvp(T(X, dev), 1024, 53)
    oud, ouv, _, _ = oracle_mod.Oracle(sc).jvp(X, 1024, 54)
    for j in (0, 1, 2, 21):
        print(parity(ud.cpu().numpy()[:, j], _se(uv.cpu().numpy()[:, j]), oud[:, j], _se(ouv[:, j]),
                     name=f"inflation du/dpi_{j} fp32"))
    # one monopole: u = r0^2 - r^2, du/da = 2a/c^2, du/dp = 2(x - p)
    p, a, c = (0.1, -0.2), 0.5, -1.0
    X, r = _disk_points(128, 15, p, 0.45)
    one = dwos.Solver.from_scene(scenes.monopole_scene([[a, *p]], c=c, src_c0=4.0, eps=1e-4, delta=1e-3), "fp32")
    m, v = one.solve(T(X, dev), 16384, 55)
    check_vs_exact(m.cpu().numpy(), _se(v.cpu().numpy()), (a / -c) ** 2 - r ** 2, 3e-4, "monopole Poisson fp32")
    # a thin shell (eps = delta / 100): the nested walks' shell bias, about
    # -eps |du/dn| / delta relative, stays well under the budget
    one = dwos.Solver.from_scene(scenes.monopole_scene([[a, *p]], c=c, src_c0=4.0, eps=1e-4, delta=1e-2), "fp32")
    ud, uv, _ = one.jvp(T(X, dev), 16384, 56)
    ud, se = ud.cpu().numpy(), _se(uv.cpu().numpy())
    check_vs_exact(ud[:, 0], se[:, 0], np.full(len(X), 2 * a / c ** 2), 0.03, "du/da fp32")
    check_vs_exact(ud[:, 1], se[:, 1], 2 * (X[:, 0] - p[0]), 0.03, "du/dpx fp32")
    check_vs_exact(ud[:, 2], se[:, 2], 2 * (X[:, 1] - p[1]), 0.03, "du/dpy fp32")


def test_reverse_mode_is_weighted_forward_mode_fp32(dev, dwos):
    sc = scenes.inflation_scene(32, seed=17)
    X = T(_inside(sc.mono, sc.mono_c, 300, 18), dev)
    w = np.random.default_rng(19).normal(size=300)
    s = dwos.Solver.from_scene(sc, "fp32")
    ud, _, _ = s.jvp(X, 64, 61, var=False)
    g, _ = s.grad(X, T(w, dev), 64, 61)
    ref = (T(w, dev)[:, None] * ud).sum(0)
    assert np.allclose(g.cpu().numpy(), ref.cpu().numpy(), rtol=1e-9, atol=1e-9 * float(ref.abs().max()))


# ------------------------------------------------------------- error paths --

def test_implicit_error_paths(dev, dwos):
    from paper_2405_12964_amd.capi import DwosError, DWOS_EINVAL, DWOS_ESTATE
    good = np.array([[0.5, 0.0, 0.0]])
    for mono, c in ((np.array([[0.0, 0, 0]]), -1.0), (np.array([[-0.1, 0, 0]]), -1.0), (good, 0.0),
                    (good, 1.0), (np.array([[0.5, np.nan, 0]]), -1.0), (np.zeros((1025, 3)) + [0.1, 0, 0], -1.0)):
        with pytest.raises(DwosError) as e:
            dwos.Solver(2, "fp32").set_implicit(mono, c)
        assert e.value.code == DWOS_EINVAL
    with pytest.raises(DwosError) as e:
        dwos.Solver(3, "fp32").set_implicit(good, -1.0)
    assert e.value.code == DWOS_EINVAL
    # a mesh boundary and an implicit one exclude each other
    s = dwos.Solver(2, "fp32")
    s.set_boundary(np.array([[0.0, 0], [1, 0], [0, 1]]), np.array([[0, 1], [1, 2], [2, 0]]))
    with pytest.raises(DwosError) as e:
        s.set_implicit(good, -1.0)
    assert e.value.code == DWOS_ESTATE
    s = dwos.Solver.from_scene(scenes.monopole_scene(good, src_c0=4.0), "fp32")
    with pytest.raises(DwosError) as e:
        s.set_boundary(np.array([[0.0, 0], [1, 0], [0, 1]]), np.array([[0, 1], [1, 2], [2, 0]]))
    assert e.value.code == DWOS_ESTATE
    with pytest.raises(DwosError) as e:
        s.set_reflecting(np.array([[0.0, 0], [1, 0]]), np.array([[0, 1]]))
    assert e.value.code == DWOS_ESTATE
    X = T([[0.1, 0.1]], dev)
    with pytest.raises(DwosError) as e:
        s.implicit_band_grad(X, T([1.0], dev), 0.0)
    assert e.value.code == DWOS_EINVAL
    # empty calls
    m, _ = s.solve(T(np.zeros((0, 2)), dev), 4, 1)
    assert m.numel() == 0
    g, _ = s.grad(T(np.zeros((0, 2)), dev), T(np.zeros(0), dev), 4, 1)
    assert np.array_equal(g.cpu().numpy(), np.zeros(3))
    # removing the implicit boundary leaves no boundary
    s.set_implicit(np.zeros((0, 3)), -1.0)
    with pytest.raises(DwosError) as e:
        s.solve(X, 4, 1)
    assert e.value.code == DWOS_ESTATE


# ------------------------------------------------------ optimisation loop --

def test_inflation_loop_reduces_loss(dev, dwos):
    """Curve inflation (Sec. 7.4) through ImplicitShapeOptimizer on a 64 x 64
    image: starting from another random blob, the image loss against the
    target's heightfield falls, and every iteration's walks stay valid."""
    from paper_2405_12964_amd.shapeopt import ImplicitShapeOptimizer
    side = 64
    g1 = -1.0 + (np.arange(side) + 0.5) * 2.0 / side
    Xt = T(np.stack(np.meshgrid(g1, g1), -1).reshape(-1, 2), dev)
    dA, eps_band = (2.0 / side) ** 2, 4.0 / side
    target = scenes.inflation_scene(32, seed=1).with_(K=4)
    ref = dwos.Solver.from_scene(target, "fp32")
    _, reg = ref.implicit_band_grad(Xt, torch.zeros(len(Xt), dtype=torch.float64, device=dev), eps_band,
                                    want_mask=True)
    inside = torch.nonzero(reg > 0).squeeze(1)
    uref = torch.zeros(len(Xt), dtype=torch.float64, device=dev)
    uref[inside] = ref.solve(Xt[inside].contiguous(), 256, 99)[0]
    opt = ImplicitShapeOptimizer(scenes.inflation_scene(32, seed=2).with_(K=4), Xt, uref, dA, eps_band,
                                 lr=5e-3, W=8)
    opt.solver.walk_timing(0, reset=True)
    opt.solver.walk_timing(1, reset=True)
    hist = [opt.step(1000 + i) for i in range(60)]
    losses = [h[0] for h in hist]
    for k in (0, 1):
        assert opt.solver.walk_timing(k)[2]["invalid"] == 0
    assert np.all(opt.mono[:, 0] >= 1e-3)
    first, last = np.mean(losses[:5]), np.mean(losses[-5:])
    print(f"inflation loss: first 5 iterations {first:.4e}, last 5 {last:.4e}; pixels inside "
          f"{[h[1] for h in hist[::10]]}")
    assert np.all(np.isfinite(losses)) and last < 0.7 * first, (first, last)
