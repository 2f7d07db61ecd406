"""Walk on stars with a Robin condition on the reflecting boundary (Sec. 3.4,
eq. (mixed_bvp): du/dn - mu u = h, n into the domain) and its differential
version (Sec. 4.4, eq. (mixed_bvp_deriv)) on the GPU, through the C ABI.

* Walk for walk: the FP64 instantiation reproduces every oracle walk (u with
  the Robin data terms and the throughput's signs, query counts, terminal
  primitive, nested mean, udot) within 1e-9, from inside and from wall
  points, forward and differential.
* FP32 against closed forms: the half disk's harmonic field with Robin data
  on its diameter, the Robin annulus (values and du/da).
* FP32 against the oracle under the parity rule (independent seeds); reverse
  mode equals the weighted forward mode (the throughput enters both).
* Error paths of dwos_set_robin.
"""
import numpy as np
import pytest
from scipy import special

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


def T(x, dev):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=dev)


def _se(v):
    return np.sqrt(np.maximum(np.asarray(v, float), 0))


def _half_disk(mu, **kw):
    sc = scenes.half_disk_scene(g="x2-y2+y", **kw)
    return sc.with_(robin_mu=mu, robin_h=scenes._restricted(1.0, None, [[-mu, 0.0], [0.0, 0.0]], 2))


def _field(X):
    return X[:, 0] ** 2 - X[:, 1] ** 2 + X[:, 1]


def _annulus(a=0.4, b=1.0, k=2.0, mu=0.8, h=0.3, **kw):
    return scenes.annulus_reflecting_scene(a, b, sigma=k * k, **kw).with_(
        robin_mu=mu, robin_h=scenes._restricted(h, dim=2))


def _annulus_exact(a, b, k, mu, h, ga=1.0):
    if k == 0:
        f, fp = (lambda r: np.ones_like(r)), (lambda r: np.zeros_like(r))
        g, gp = (lambda r: np.log(r)), (lambda r: 1.0 / r)
    else:
        f, fp = (lambda r: special.i0(k * r)), (lambda r: k * special.i1(k * r))
        g, gp = (lambda r: special.k0(k * r)), (lambda r: -k * special.k1(k * r))
    A = np.array([[f(np.array(a)), g(np.array(a))],
                  [-fp(np.array(b)) - mu * f(np.array(b)), -gp(np.array(b)) - mu * g(np.array(b))]], float)
    c = np.linalg.solve(A, [ga, h])
    return lambda r: c[0] * f(r) + c[1] * g(r)


def _annulus_points(n, seed, a=0.4, b=1.0):
    rng = np.random.default_rng(seed)
    r = rng.uniform(a + 0.05, b - 0.05, n)
    t = rng.uniform(0, 2 * np.pi, n)
    return np.stack([r * np.cos(t), r * np.sin(t)], 1), r


def _wfw(dev, dwos, oracle_mod, sc, X, W, seed, modes=(0, 1), start=None):
    s = dwos.Solver.from_scene(sc, "fp64")
    o = oracle_mod.Oracle(sc)
    if start is not None:
        s.set_start_segments(start)
    Xt = T(X, dev)
    for mode in modes:
        g = s.walk_records(Xt, W, seed, mode=mode, udot=(mode == 1 and sc.N > 0))
        r = o.walk_records(X, W, seed, mode=mode, start_seg=start)
        gu = g["u"].cpu().numpy()
        # relative to the walk's size: a Robin walk's throughput can grow
        # large (its weights exceed 1 and flip sign; the rounding of the
        # two builds then differs in the last digits of a large value)
        close = np.abs(gu - r["u"]) <= 1e-9 * np.maximum(1.0, np.abs(r["u"]))
        assert close.all(), (mode, np.abs(gu - r["u"]).max())
        assert np.array_equal(g["steps"].cpu().numpy(), r["steps"]), mode
        if mode == 1:
            assert np.array_equal(g["prim"].cpu().numpy(), r["prim"])
            go = g["uoff"].cpu().numpy()
            assert (np.abs(go - r["uoff"]) <= 1e-9 * np.maximum(1.0, np.abs(r["uoff"]))).all()
            gd = g["udot"].cpu().numpy()
            close = np.abs(gd - r["udot"]) <= 1e-9 * np.maximum(1.0, np.abs(r["udot"]))
            assert close.all(), np.abs(gd - r["udot"]).max()
    return s


@pytest.mark.parametrize("mu", [0.0, 0.7])
def test_walk_for_walk_half_disk_robin(dev, dwos, oracle_mod, mu):
    sc = _half_disk(mu, eps=1e-3, delta=1e-2)
    Xw, seg = scenes.points_on_segments(sc.NV, sc.nsegs, 8, 81)
    Xi = scenes.points_in_half_disk(8, 82)
    X = np.concatenate([Xw, Xi])
    start = np.concatenate([seg, -np.ones(8, np.int32)])
    _wfw(dev, dwos, oracle_mod, sc, X, 16, 83, start=start)


def test_walk_for_walk_annulus_robin(dev, dwos, oracle_mod):
    sc = _annulus(n_in=64, n_out=128, eps=1e-3, delta=1e-2, K=2)
    X, _ = _annulus_points(12, 84)
    _wfw(dev, dwos, oracle_mod, sc, X, 16, 85)
    # Laplace with a stronger Robin coefficient (weights beyond 1 and sign
    # flips in the throughput, which then grows large on some walks)
    sc = _annulus(k=0.0, mu=3.0, h=-0.5, n_in=64, n_out=128, eps=1e-3, delta=1e-2)
    _wfw(dev, dwos, oracle_mod, sc, X, 16, 86)


def test_fp32_closed_forms(dev, dwos):
    mu = 0.7
    sc = _half_disk(mu, eps=1e-4, delta=1e-3)
    s = dwos.Solver.from_scene(sc, "fp32")
    X = scenes.points_in_half_disk(256, 87, rmax=0.9)
    m, v = s.solve(T(X, dev), 16384, 88)
    check_vs_exact(m.cpu().numpy(), _se(v.cpu().numpy()), _field(X), 4e-4, "half disk Robin fp32")
    Xw, seg = scenes.points_on_segments(sc.NV, sc.nsegs, 256, 89)
    keep = np.abs(Xw[:, 0]) < 0.9
    Xw, seg = Xw[keep], seg[keep]
    s.set_start_segments(seg)
    m, v = s.solve(T(Xw, dev), 16384, 90)
    s.set_start_segments(None)
    check_vs_exact(m.cpu().numpy(), _se(v.cpu().numpy()), _field(Xw), 4e-4, "half disk Robin fp32 wall")
    a, b, k, mu, h = 0.4, 1.0, 2.0, 0.8, 0.3
    sc = _annulus(a, b, k, mu, h, eps=1e-3, delta=1e-2)
    X, r = _annulus_points(128, 91)
    s = dwos.Solver.from_scene(sc, "fp32")
    m, v = s.solve(T(X, dev), 16384, 92)
    check_vs_exact(m.cpu().numpy(), _se(v.cpu().numpy()), _annulus_exact(a, b, k, mu, h)(r), 5e-4,
                   "annulus Robin fp32")
    ud, uv, _ = s.jvp(T(X, dev), 16384, 93)
    e = 1e-6
    du = (_annulus_exact(a + e, b, k, mu, h)(r) - _annulus_exact(a - e, b, k, mu, h)(r)) / (2 * e)
    check_vs_exact(ud.cpu().numpy()[:, 0], _se(uv.cpu().numpy()[:, 0]), du, 0.05 * np.abs(du).max(),
                   "annulus Robin du/da fp32")


def test_fp32_parity_with_oracle(dev, dwos, oracle_mod):
    sc = _annulus(n_in=128, n_out=256, eps=1e-3, delta=1e-2)
    X, _ = _annulus_points(48, 94)
    s = dwos.Solver.from_scene(sc, "fp32")
    m, v = s.solve(T(X, dev), 2048, 95)
    om, ov, _ = oracle_mod.Oracle(sc).solve(X, 2048, 96)
    print(parity(m.cpu().numpy(), _se(v.cpu().numpy()), om, _se(ov), name="annulus Robin solve"))
    ud, uv, _ = s.jvp(T(X, dev), 2048, 97)
    oud, ouv, _, _ = oracle_mod.Oracle(sc).jvp(X, 2048, 98)
    print(parity(ud.cpu().numpy()[:, 0], _se(uv.cpu().numpy()[:, 0]), oud[:, 0], _se(ouv[:, 0]),
                 name="annulus Robin jvp"))


def test_reverse_mode_is_weighted_forward_mode(dev, dwos):
    sc = _annulus(k=0.0, mu=3.0, h=-0.5, n_in=128, n_out=256, eps=1e-3, delta=1e-2)
    X, _ = _annulus_points(256, 99)
    Xt = T(X, dev)
    w = np.random.default_rng(100).normal(size=len(X))
    for prec in ("fp64", "fp32"):
        s = dwos.Solver.from_scene(sc, prec)
        ud, _, _ = s.jvp(Xt, 512, 21, var=False)
        g, _ = s.grad(Xt, T(w, dev), 512, 21)
        ref = (T(w, dev)[:, None] * ud).sum(0)
        assert np.allclose(g.cpu().numpy(), ref.cpu().numpy(), rtol=1e-9, atol=1e-9 * float(ref.abs().max()))


def test_robin_error_paths(dev, dwos):
    from paper_2405_12964_amd.capi import DwosError, DWOS_EINVAL, DWOS_ESTATE
    s = dwos.Solver.from_scene(scenes.c1_polygon(32), "fp32")
    with pytest.raises(DwosError) as e:
        s.set_robin(0.5)
    assert e.value.code == DWOS_ESTATE
    s.set_robin(0.0)   # zero flux without a reflecting boundary: nothing to set
    s2 = dwos.Solver.from_scene(_annulus(n_in=32, n_out=64), "fp32")
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(DwosError) as e:
            s2.set_robin(bad)
        assert e.value.code == DWOS_EINVAL
    with pytest.raises(DwosError) as e:
        s2.set_robin(1.0, dict(kind="mapped"))
    assert e.value.code == DWOS_EINVAL
