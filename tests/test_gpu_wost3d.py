"""Walk on stars over 3D reflecting triangle meshes on the GPU against the
FP64 oracle, through the C ABI.

* The two reflecting-mesh queries (closest silhouette edge, first triangle
  hit along a ray) equal the oracle's, from inside and from wall points.
* Walk for walk: the FP64 instantiation of the 3D walk-on-stars kernel
  reproduces every oracle walk (u, query counts, terminal primitive, nested
  mean, udot) within 1e-9: the L-shaped prism (Laplace and screened), walks
  from its walls, the cube's Robin wall, and the half ball's differential
  walks with their nested walks.
* Statistical: the FP32 path against the oracle (independent seeds) and
  against closed forms (the re-entrant edge, the Robin wall, the half
  ball's radius derivative); reverse mode equals the weighted forward mode.
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


def T(x, dev, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device=dev)


def _se(v):
    return np.sqrt(np.maximum(np.asarray(v, float), 0))


def _cyl(X):
    return np.hypot(X[:, 0], X[:, 1]), np.mod(np.arctan2(X[:, 1], X[:, 0]), 2 * np.pi)


def _screened_edge(k):
    return lambda r, th: special.iv(2.0 / 3.0, k * r) * np.cos(2 * th / 3)


def _robin_cube(n_wall=3, mu=0.5):
    """u = 1 + x/2 + x^2 - z^2 with du/dn - mu u = h on the wall x = -1."""
    g = scenes._restricted(1.0, [0.5, 0.0, 0.0], np.diag([1.0, 0.0, -1.0]), 3)
    h = scenes._restricted(-1.5 - mu * 1.5, None, np.diag([0.0, 0.0, mu]), 3)
    return scenes.box_wall_scene(n_wall=n_wall, g=g, robin_mu=mu, robin_h=h, graded=2.0)


def _dirs(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# ------------------------------------------------------------------ queries --

def _query_cases(sc, Xi, seed):
    rng = np.random.default_rng(seed)
    Xw, tri = scenes.points_on_triangles(sc.NV, sc.nsegs, 150, seed + 1)
    a, b, c = (sc.NV[sc.nsegs[tri, k]] for k in range(3))
    nin = np.cross(b - a, c - a)
    nin /= np.linalg.norm(nin, axis=1, keepdims=True)
    X = np.concatenate([Xi, Xw])
    D = _dirs(rng, len(X))
    on = np.concatenate([-np.ones(len(Xi), np.int32), tri]).astype(np.int32)
    N = np.concatenate([np.zeros((len(Xi), 3)), nin])
    cdot = np.sum(D * N, 1)
    flip = (on >= 0) & (cdot < 0)
    D[flip] -= 2 * cdot[flip, None] * N[flip]
    cap = rng.uniform(0.2, 3.0, len(X))
    return X, D, cap, on, N


@pytest.mark.parametrize("name", ["lprism", "half_ball"])
def test_reflect_queries_3d_match_oracle(dev, dwos, oracle_mod, name):
    if name == "lprism":
        sc = scenes.lprism_scene(n=4, n_wall=6)
        Xi = scenes.points_in_lprism(200, 3, zlim=0.9)
    else:
        sc = scenes.half_ball_scene()
        Xi = scenes.points_in_half_ball(200, 3, rmax=0.95)
    X, D, cap, on, N = _query_cases(sc, Xi, 7)
    o = oracle_mod.Oracle(sc)
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
        tol = 1e-9 * np.maximum(1.0, np.abs(r["u"]))
        assert np.all(np.abs(gu - r["u"]) <= tol), (mode, np.abs(gu - r["u"]).max())
        assert np.array_equal(g["steps"].cpu().numpy(), r["steps"]), mode
        if mode == 1:
            assert np.array_equal(g["prim"].cpu().numpy(), r["prim"])
            assert np.allclose(g["uoff"].cpu().numpy(), r["uoff"], rtol=1e-9, atol=1e-9)
            if sc.N > 0:
                gd = g["udot"].cpu().numpy()
                scale = max(1.0, float(np.abs(r["udot"]).max()))
                assert np.allclose(gd, r["udot"], rtol=0, atol=1e-9 * scale), np.abs(gd - r["udot"]).max()


def test_walk_for_walk_lprism(dev, dwos, oracle_mod):
    X = scenes.points_in_lprism(10, 1, zlim=0.6)
    _wfw(dev, dwos, oracle_mod, scenes.lprism_scene(n=4, n_wall=4), X, 8, 11, modes=(0,))
    k = 2.0
    sc = scenes.lprism_scene(n=4, n_wall=4, sigma=k * k, gfun=_screened_edge(k))
    _wfw(dev, dwos, oracle_mod, sc, X, 8, 12, modes=(0,))


def test_walk_for_walk_from_the_walls_3d(dev, dwos, oracle_mod):
    sc = scenes.lprism_scene(n=4, n_wall=4)
    X, tri = scenes.points_on_triangles(sc.NV, sc.nsegs, 8, 2)
    Xi = scenes.points_in_lprism(4, 4, zlim=0.6)
    X = np.concatenate([X, Xi])
    tri = np.concatenate([tri, -np.ones(4, np.int32)])
    _wfw(dev, dwos, oracle_mod, sc, X, 8, 13, modes=(0,), start=tri)


def test_walk_for_walk_robin_wall(dev, dwos, oracle_mod):
    X = np.random.default_rng(5).uniform(-0.85, 0.85, (10, 3))
    _wfw(dev, dwos, oracle_mod, _robin_cube(), X, 8, 14, modes=(0,))


def test_walk_for_walk_half_ball_derivatives(dev, dwos, oracle_mod):
    sc = scenes.half_ball_scene(n_az=24, n_pol=6, n_rad=6, g="one", sigma=4.0, eps=1e-3, delta=1e-2, K=2)
    _wfw(dev, dwos, oracle_mod, sc, scenes.points_in_half_ball(8, 6), 8, 15)
    sc = scenes.half_ball_scene(n_az=24, n_pol=6, n_rad=6, g="x2-z2", eps=1e-3, delta=1e-2).with_(src_c0=3.0)
    _wfw(dev, dwos, oracle_mod, sc, scenes.points_in_half_ball(8, 7), 8, 16)


def test_walk_for_walk_closed_reflecting_surface(dev, dwos, oracle_mod):
    """The 3D thermal stand-in at a small size (a closed, convex-ish
    reflecting superellipsoid of 720 triangles between four heating
    elements): the silhouette query prunes edge-BVH children by their normal
    cones, the oracle tests every edge; walks from the slice surface and from
    the gap, forward and differential with the elements' shape derivatives."""
    sc = scenes.thermal3d_scene(nu_slice=6, nu_wire=3, eps=1e-3, delta=1e-2, K=2)
    X, tri = scenes.points_on_triangles(sc.NV, sc.nsegs, 8, 17)
    Xi = np.array([[1.1, 0.0, 0.0], [-1.1, 0.2, 0.1], [0.0, 0.9, 0.3], [0.3, -0.2, 0.9]])
    X = np.concatenate([X, Xi])
    tri = np.concatenate([tri, -np.ones(len(Xi), np.int32)])
    _wfw(dev, dwos, oracle_mod, sc, X, 8, 18, start=tri)


def test_staged_edge_tree_same_walks(dev, dwos):
    """FP32 walk on stars reads the edge BVH's first nodes and cones from
    LDS: with the staging switched off (stage_nodes = 0) every walk is the
    same, value and step count, forward and differential."""
    sc = scenes.thermal3d_scene(nu_slice=24, nu_wire=3, K=2)
    X, tri = scenes.points_on_triangles(sc.NV, sc.nsegs, 256, 23)
    s = dwos.Solver.from_scene(sc, "fp32")
    s.set_start_segments(tri)
    out = {}
    for cap in (-1, 0):
        s.set_tuning(stage_nodes=cap)
        out[cap] = [s.walk_records(T(X, dev), 16, 31, mode=mode) for mode in (0, 1)]
    for r0, r1 in zip(out[-1], out[0]):
        for key in ("u", "steps"):
            assert torch.equal(r0[key], r1[key]), key
    assert int(out[0][0]["steps"].max()) > 10


def test_silhouette_cones_match_oracle(dev, dwos, oracle_mod):
    """Closest silhouette edge of the closed slice from points around it
    (off the surface and on it): the cone-pruned query equals the oracle's
    full search, exactly in FP64.  In FP32 an edge that is within the edge-on
    tolerance (1e-4 of its operands) counts as a silhouette seen from a point
    off the surface, so the FP32 distance may be shorter than the oracle's
    (never longer: the star region stays star-shaped) for a few points."""
    sc = scenes.thermal3d_scene(nu_slice=10, nu_wire=2)
    rng = np.random.default_rng(19)
    U = rng.normal(size=(300, 3))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    Xi = U * rng.uniform(1.02, 1.8, (300, 1)) * np.array([0.9, 0.6, 0.6])
    X, D, cap, on, N = _query_cases(sc, Xi, 20)
    o = oracle_mod.Oracle(sc)
    ref = np.array([o.silhouette(X[i], int(on[i]), N[i], cap[i]) for i in range(len(X))])
    for prec, tol in (("fp64", 1e-12), ("fp32", 2e-5)):
        s = dwos.Solver.from_scene(sc, prec)
        out = s.reflect_query(T(X, dev), T(D, dev), T(cap, dev), T(on, dev, torch.int32), T(N, dev)).cpu().numpy()
        close = np.isclose(out[:, 0], ref, rtol=tol, atol=tol * 0.1)
        if prec == "fp64":
            assert close.all(), (prec, np.abs(out[:, 0] - ref).max())
        else:
            assert np.all(out[:, 0] <= ref * (1 + tol) + tol * 0.1), (out[:, 0] - ref).max()
            assert close.mean() > 0.99, (close.mean(), np.abs(out[:, 0] - ref).max())


# ------------------------------------------------- FP32 statistical parity --

def test_fp32_parity_3d(dev, dwos, oracle_mod):
    k = 2.0
    sc = scenes.lprism_scene(n=4, n_wall=4, sigma=k * k, gfun=_screened_edge(k))
    X = scenes.points_in_lprism(32, 8, zlim=0.6)
    m, v = dwos.Solver.from_scene(sc, "fp32").solve(T(X, dev), 1024, 101)
    om, ov, _ = oracle_mod.Oracle(sc).solve(X, 512, 202)
    print(parity(m.cpu().numpy(), _se(v.cpu().numpy()), om, _se(ov * 2), name="L-prism screened"))
    sc = _robin_cube()
    X = np.random.default_rng(9).uniform(-0.85, 0.85, (32, 3))
    m, v = dwos.Solver.from_scene(sc, "fp32").solve(T(X, dev), 1024, 103)
    om, ov, _ = oracle_mod.Oracle(sc).solve(X, 512, 204)
    print(parity(m.cpu().numpy(), _se(v.cpu().numpy()), om, _se(ov * 2), name="Robin cube"))
    sc = scenes.half_ball_scene(g="one", sigma=4.0, eps=1e-3, delta=1e-2)
    X = scenes.points_in_half_ball(32, 10, rmax=0.7)
    ud, uv, _ = dwos.Solver.from_scene(sc, "fp32").jvp(T(X, dev), 1024, 105)
    oud, ouv, _, _ = oracle_mod.Oracle(sc).jvp(X, 512, 206)
    print(parity(ud.cpu().numpy()[:, 0], _se(uv.cpu().numpy()[:, 0]), oud[:, 0], _se(ouv[:, 0] * 2),
                 name="half ball jvp"))


def test_fp32_closed_forms_3d(dev, dwos):
    """The re-entrant edge (screened) from inside and from the walls, the
    Robin wall, and the half ball's radius derivative, at many walks."""
    k = 2.0
    g = _screened_edge(k)
    sc = scenes.lprism_scene(n=6, n_wall=6, sigma=k * k, gfun=g)
    s = dwos.Solver.from_scene(sc, "fp32")
    X = scenes.points_in_lprism(128, 10, zlim=0.4)
    m, v = s.solve(T(X, dev), 16384, 105)
    check_vs_exact(m.cpu().numpy(), _se(v.cpu().numpy()), g(*_cyl(X)), 3e-3, "L-prism fp32")
    Xw, tri = scenes.points_on_triangles(sc.NV, sc.nsegs, 128, 11)
    keep = np.abs(Xw[:, 2]) < 0.6   # away from the caps' interpolated data
    Xw, tri = Xw[keep], tri[keep]
    s.set_start_segments(tri)
    m, v = s.solve(T(Xw, dev), 16384, 106)
    s.set_start_segments(None)
    check_vs_exact(m.cpu().numpy(), _se(v.cpu().numpy()), g(*_cyl(Xw)), 3e-3, "L-prism fp32 walls")
    sc = _robin_cube()
    X = np.random.default_rng(12).uniform(-0.85, 0.85, (128, 3))
    m, v = dwos.Solver.from_scene(sc, "fp32").solve(T(X, dev), 16384, 107)
    u = 1 + 0.5 * X[:, 0] + X[:, 0] ** 2 - X[:, 2] ** 2
    check_vs_exact(m.cpu().numpy(), _se(v.cpu().numpy()), u, 1e-3, "Robin cube fp32")
    sc = scenes.half_ball_scene(g="one", sigma=k * k, eps=1e-3, delta=1e-2)
    X = scenes.points_in_half_ball(64, 13, rmax=0.7)
    r = np.linalg.norm(X, axis=1)
    ud, uv, _ = dwos.Solver.from_scene(sc, "fp32").jvp(T(X, dev), 16384, 108)
    exact = np.sinh(k * r) / (r * np.sinh(k)) * (1 - k / np.tanh(k))
    check_vs_exact(ud.cpu().numpy()[:, 0], _se(uv.cpu().numpy()[:, 0]), exact, 0.06 * np.abs(exact).max(),
                   "half ball du/dR fp32")


def test_reverse_mode_is_weighted_forward_mode_3d(dev, dwos):
    sc = scenes.half_ball_scene(g="one", sigma=4.0, eps=1e-3, delta=1e-2)
    rng = np.random.default_rng(13)
    X = T(scenes.points_in_half_ball(128, 14), dev)
    w = rng.normal(size=128)
    for prec in ("fp64", "fp32"):
        s = dwos.Solver.from_scene(sc, prec)
        ud, _, _ = s.jvp(X, 256, 21, var=False)
        g, _ = s.grad(X, T(w, dev), 256, 21)
        ref = (T(w, dev)[:, None] * ud).sum(0)
        assert np.allclose(g.cpu().numpy(), ref.cpu().numpy(), rtol=1e-9, atol=1e-9 * float(ref.abs().max()))


def test_reflecting_3d_error_paths(dev, dwos):
    from paper_2405_12964_amd.capi import DwosError, DWOS_EINVAL
    sc = scenes.lprism_scene(n=4, n_wall=4)
    s = dwos.Solver.from_scene(sc, "fp32")
    with pytest.raises(DwosError) as e:
        s.set_start_segments(np.array([len(sc.nsegs)] * 4, np.int32))
    assert e.value.code == DWOS_EINVAL
    with pytest.raises(DwosError) as e:
        s.set_reflecting(sc.NV, np.array([[0, 0, 1]]))
    assert e.value.code == DWOS_EINVAL
    s.set_reflecting(np.zeros((0, 3)), np.zeros((0, 3), np.int32))
    s.solve(T(scenes.points_in_lprism(8, 1), dev), 16, 1)
