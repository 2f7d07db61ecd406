"""Walk on stars (reflecting boundaries) on the GPU against the FP64 oracle,
through the C ABI.

* The step weight and the two reflecting-boundary queries (closest
  silhouette vertex, first ray hit) equal the oracle's.
* Walk-for-walk: the FP64 instantiation of the walk-on-stars kernel
  reproduces every oracle walk (u, query counts, terminal primitive, nested
  mean, udot) within 1e-9, from inside and from reflecting start points.
* Statistical: the FP32 path against the oracle (independent seeds) and
  against closed forms; reverse mode equals the weighted forward mode.
* Error paths of the entry points.
"""
import math

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


def T(x, dev, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device=dev)


def _se(v):
    return np.sqrt(np.maximum(np.asarray(v, float), 0))


def _polar(X):
    return np.hypot(X[:, 0], X[:, 1]), np.mod(np.arctan2(X[:, 1], X[:, 0]), 2 * np.pi)


def _screened_corner(k):
    return lambda r, th: special.iv(2.0 / 3.0, k * r) * np.cos(2 * th / 3)


# ------------------------------------------------------- weight and queries --

def test_reflect_weight_matches_oracle(dev, dwos, oracle_mod):
    rng = np.random.default_rng(1)
    R = np.exp(rng.uniform(np.log(1e-3), np.log(3.0), 400))
    r = np.clip(rng.uniform(0, 1, 400), 1e-6, 1.0) * R
    for D in (2, 3):
        for sigma in (0.0, 0.5, 4.0, 40.0, 900.0):
            ref = np.array([oracle_mod.neumann_weight(D, sigma, a, b) for a, b in zip(r, R)])
            for prec, tol in (("fp64", 1e-11), ("fp32", 2e-5)):
                w = dwos.Solver(D, prec).eval_reflect_weight(T(r, dev), T(R, dev), sigma).cpu().numpy()
                assert np.allclose(w, ref, rtol=tol, atol=0), (D, sigma, prec, np.abs(w / ref - 1).max())


def _queries(sc, X, D, cap, on, nin):
    return dict(X=X, dirs=D, cap=cap, on=on, nin=nin)


def _query_cases(sc, seed):
    """Interior points with random directions, and wall points (with their
    domain side) with directions into the domain."""
    rng = np.random.default_rng(seed)
    if sc.name == "lshape":
        Xi = scenes.points_in_lshape(300, seed)
    else:
        Xi = scenes.points_in_half_disk(300, seed)
    Xw, seg = scenes.points_on_segments(sc.NV, sc.nsegs, 200, seed + 1)
    a, b = sc.NV[sc.nsegs[seg, 0]], sc.NV[sc.nsegs[seg, 1]]
    t = b - a
    nin = np.stack([-t[:, 1], t[:, 0]], 1) / np.linalg.norm(t, axis=1)[:, None]
    X = np.concatenate([Xi, Xw])
    ang = rng.uniform(0, 2 * np.pi, len(X))
    D = np.stack([np.cos(ang), np.sin(ang)], 1)
    on = np.concatenate([-np.ones(len(Xi), np.int32), seg]).astype(np.int32)
    N = np.concatenate([np.zeros((len(Xi), 2)), nin])
    # wall points look into the domain
    c = np.sum(D * N, 1)
    flip = (on >= 0) & (c < 0)
    D[flip] -= 2 * c[flip, None] * N[flip]
    cap = rng.uniform(0.2, 3.0, len(X))
    return X, D, cap, on, N


@pytest.mark.parametrize("name", ["lshape", "half_disk"])
def test_reflect_queries_match_oracle(dev, dwos, oracle_mod, name):
    sc = scenes.lshape_scene() if name == "lshape" else scenes.half_disk_scene()
    X, D, cap, on, N = _query_cases(sc, 7)
    o = oracle_mod.Oracle(sc)
    # as in a walk step, the reach is within the Dirichlet distance (rays
    # then stay in the domain and meet walls from their domain side)
    cap = np.minimum(cap, [o.closest(x)["d"] for x in X])
    ref = np.zeros((len(X), 3))
    for i in range(len(X)):
        ref[i, 0] = o.silhouette(X[i], int(on[i]), N[i], cap[i])
        ref[i, 1:] = o.ray(X[i], D[i], cap[i], int(on[i]))
    for prec in ("fp64", "fp32"):
        s = dwos.Solver.from_scene(sc, prec)
        out = s.reflect_query(T(X, dev), T(D, dev), T(cap, dev), T(on, dev, torch.int32), T(N, dev)).cpu().numpy()
        if prec == "fp64":
            assert np.allclose(out[:, 0], ref[:, 0], rtol=1e-12, atol=1e-14), np.abs(out[:, 0] - ref[:, 0]).max()
            assert np.array_equal(out[:, 2].astype(int), ref[:, 2].astype(int))
            assert np.allclose(out[:, 1], ref[:, 1], rtol=1e-12, atol=1e-14)
        else:
            assert np.allclose(out[:, 0], ref[:, 0], rtol=2e-5, atol=2e-6)
            same = out[:, 2].astype(int) == ref[:, 2].astype(int)
            assert same.mean() > 0.98
            assert np.allclose(out[same, 1], ref[same, 1], rtol=2e-5, atol=2e-6)
    # invalid segment index: NaN row, no fault
    bad = np.array([len(sc.nsegs) + 5], np.int32)
    out = dwos.Solver.from_scene(sc, "fp64").reflect_query(
        T(X[:1], dev), T(D[:1], dev), T(cap[:1], dev), T(bad, dev, torch.int32), T(N[:1], dev)).cpu().numpy()
    assert np.all(np.isnan(out))


# ------------------------------------------------------------ walk for walk --

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
        assert np.allclose(gu, r["u"], rtol=0, atol=1e-9), (mode, np.abs(gu - r["u"]).max())
        assert np.array_equal(g["steps"].cpu().numpy(), r["steps"]), mode
        if mode == 1:
            assert np.array_equal(g["prim"].cpu().numpy(), r["prim"])
            assert np.allclose(g["uoff"].cpu().numpy(), r["uoff"], rtol=0, atol=1e-9)
            if sc.N > 0:
                gd = g["udot"].cpu().numpy()
                scale = max(1.0, float(np.abs(r["udot"]).max()))
                assert np.allclose(gd, r["udot"], rtol=0, atol=1e-9 * scale), np.abs(gd - r["udot"]).max()


def test_walk_for_walk_lshape(dev, dwos, oracle_mod):
    X = scenes.points_in_lshape(16, 1)
    _wfw(dev, dwos, oracle_mod, scenes.lshape_scene(), X, 16, 11, modes=(0,))
    k = 2.0
    sc = scenes.lshape_scene(sigma=k * k, gfun=_screened_corner(k))
    _wfw(dev, dwos, oracle_mod, sc, X, 16, 12, modes=(0,))


def test_walk_for_walk_from_the_wall(dev, dwos, oracle_mod):
    sc = scenes.lshape_scene()
    X, seg = scenes.points_on_segments(sc.NV, sc.nsegs, 12, 2)
    _wfw(dev, dwos, oracle_mod, sc, X, 16, 13, modes=(0,), start=seg)
    sc = scenes.half_disk_scene(sigma=4.0, g="one", eps=1e-3, delta=1e-2)
    X, seg = scenes.points_on_segments(sc.NV, sc.nsegs, 12, 3)
    # a mix of wall and interior points
    Xi = scenes.points_in_half_disk(4, 4)
    X = np.concatenate([X, Xi])
    seg = np.concatenate([seg, -np.ones(4, np.int32)])
    _wfw(dev, dwos, oracle_mod, sc, X, 16, 14, start=seg)


def test_walk_for_walk_source_and_derivatives(dev, dwos, oracle_mod):
    sc = scenes.half_disk_scene(g="zero", sigma=9.0, eps=1e-3, delta=1e-2).with_(src_c0=9.0, K=2)
    _wfw(dev, dwos, oracle_mod, sc, scenes.points_in_half_disk(12, 5), 16, 15)
    sc = scenes.annulus_reflecting_scene(0.4, 1.0, n_in=64, n_out=128, sigma=4.0, eps=1e-3, delta=1e-2)
    rng = np.random.default_rng(6)
    r = rng.uniform(0.45, 0.95, 12)
    t = rng.uniform(0, 2 * np.pi, 12)
    _wfw(dev, dwos, oracle_mod, sc, np.stack([r * np.cos(t), r * np.sin(t)], 1), 16, 16)


# ------------------------------------------------- FP32 statistical parity --

def test_fp32_parity_solve_and_jvp(dev, dwos, oracle_mod):
    k = 2.0
    sc = scenes.lshape_scene(sigma=k * k, gfun=_screened_corner(k))
    X = scenes.points_in_lshape(64, 8)
    m, v = dwos.Solver.from_scene(sc, "fp32").solve(T(X, dev), 1024, 101)
    om, ov, _ = oracle_mod.Oracle(sc).solve(X, 1024, 202)
    print(parity(m.cpu().numpy(), _se(v.cpu().numpy()), om, _se(ov), name="L-shape screened"))
    sc = scenes.annulus_reflecting_scene(0.4, 1.0, n_in=128, n_out=256, sigma=4.0, eps=1e-3, delta=1e-2)
    rng = np.random.default_rng(9)
    r = rng.uniform(0.45, 0.95, 64)
    t = rng.uniform(0, 2 * np.pi, 64)
    X = np.stack([r * np.cos(t), r * np.sin(t)], 1)
    ud, uv, _ = dwos.Solver.from_scene(sc, "fp32").jvp(T(X, dev), 1024, 103)
    oud, ouv, _, _ = oracle_mod.Oracle(sc).jvp(X, 1024, 204)
    print(parity(ud.cpu().numpy()[:, 0], _se(uv.cpu().numpy()[:, 0]), oud[:, 0], _se(ouv[:, 0]),
                 name="annulus jvp"))


def test_fp32_closed_forms(dev, dwos):
    """Re-entrant corner (screened) from inside and from the walls, and the
    annulus inner-radius derivative, at many walks."""
    k = 2.0
    g = _screened_corner(k)
    sc = scenes.lshape_scene(sigma=k * k, gfun=g)
    s = dwos.Solver.from_scene(sc, "fp32")
    X = scenes.points_in_lshape(256, 10)
    m, v = s.solve(T(X, dev), 16384, 105)
    check_vs_exact(m.cpu().numpy(), _se(v.cpu().numpy()), g(*_polar(X)), 4e-4, "L-shape fp32")
    Xw, seg = scenes.points_on_segments(sc.NV, sc.nsegs, 256, 11)
    s.set_start_segments(seg)
    m, v = s.solve(T(Xw, dev), 16384, 106)
    s.set_start_segments(None)
    check_vs_exact(m.cpu().numpy(), _se(v.cpu().numpy()), g(*_polar(Xw)), 4e-4, "L-shape fp32 walls")
    a, b = 0.4, 1.0
    sc = scenes.annulus_reflecting_scene(a, b, sigma=k * k, eps=1e-3, delta=1e-2)
    rng = np.random.default_rng(12)
    r = rng.uniform(a + 0.05, b - 0.05, 128)
    t = rng.uniform(0, 2 * np.pi, 128)
    X = np.stack([r * np.cos(t), r * np.sin(t)], 1)
    ud, uv, um = dwos.Solver.from_scene(sc, "fp32").jvp(T(X, dev), 16384, 107)
    Nf = lambda s_: special.i0(k * s_) * special.k1(k * b) + special.k0(k * s_) * special.i1(k * b)
    dN = k * (special.i1(k * a) * special.k1(k * b) - special.k1(k * a) * special.i1(k * b))
    du = -Nf(r) / Nf(a) * dN / Nf(a)
    check_vs_exact(ud.cpu().numpy()[:, 0], _se(uv.cpu().numpy()[:, 0]), du, 0.05 * np.abs(du).max(),
                   "annulus du/da fp32")


def test_reverse_mode_is_weighted_forward_mode(dev, dwos):
    sc = scenes.annulus_reflecting_scene(0.4, 1.0, n_in=128, n_out=256, sigma=4.0, eps=1e-3, delta=1e-2)
    rng = np.random.default_rng(13)
    r = rng.uniform(0.45, 0.95, 256)
    t = rng.uniform(0, 2 * np.pi, 256)
    X = T(np.stack([r * np.cos(t), r * np.sin(t)], 1), dev)
    w = rng.normal(size=256)
    for prec in ("fp64", "fp32"):
        s = dwos.Solver.from_scene(sc, prec)
        ud, _, _ = s.jvp(X, 512, 21, var=False)
        g, _ = s.grad(X, T(w, dev), 512, 21)
        ref = (T(w, dev)[:, None] * ud).sum(0)
        assert np.allclose(g.cpu().numpy(), ref.cpu().numpy(), rtol=1e-9, atol=1e-9 * float(ref.abs().max()))


# ------------------------------------------------------------- error paths --

def test_reflecting_error_paths(dev, dwos):
    from paper_2405_12964_amd.capi import DwosError, DWOS_EINVAL, DWOS_ESTATE
    sc = scenes.lshape_scene()
    s = dwos.Solver.from_scene(sc, "fp32")
    X = T(scenes.points_in_lshape(8, 1), dev)
    # start segments: out of range, and a count that does not match the call
    with pytest.raises(DwosError) as e:
        s.set_start_segments(np.array([len(sc.nsegs)] * 8, np.int32))
    assert e.value.code == DWOS_EINVAL
    s.set_start_segments(-np.ones(4, np.int32))
    with pytest.raises(DwosError) as e:
        s.solve(X, 16, 1)
    assert e.value.code == DWOS_EINVAL
    s.set_start_segments(None)
    s.solve(X, 16, 1)
    # 3D: a degenerate reflecting triangle
    s3 = dwos.Solver(3, "fp32")
    with pytest.raises(DwosError) as e:
        s3.set_reflecting(np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0]]), np.array([[0, 1, 2]]))
    assert e.value.code == DWOS_EINVAL
    # zero-length segment
    with pytest.raises(DwosError) as e:
        s.set_reflecting(np.array([[0.0, 0.0], [0.0, 0.0]]), np.array([[0, 1]]))
    assert e.value.code == DWOS_EINVAL
    # no roulette with screening
    p = dwos.solver.make_problem(sigma=1.0, rr=0, dim=2)
    with pytest.raises(DwosError) as e:
        s.set_problem(p)
    assert e.value.code == DWOS_EINVAL
    # the control variate is not available with a reflecting boundary
    sc2 = scenes.half_disk_scene(sigma=4.0, g="one")
    s2 = dwos.Solver.from_scene(sc2, "fp32")
    net = dwos.Network(2, np.zeros((4, 2), np.float32), np.zeros(scenes.MLP_THETA_SIZE, np.float32))
    s2.attach_cv(net)
    with pytest.raises(DwosError) as e:
        s2.jvp(T(scenes.points_in_half_disk(8, 2), dev), 16, 1)
    assert e.value.code == DWOS_ESTATE
    s2.attach_cv(None)
    # removing the reflecting boundary gives back walk on spheres
    s.set_reflecting(np.zeros((0, 2)), np.zeros((0, 2), np.int32))
    s.solve(X, 16, 1)
