"""FP32 parity of the 3D walk kernel -- the shape-from-diffusion hot path,
walk_kernel<float, 3, *, *> (either launch shape) -- with the FP64 oracle, and the edge paths
of the mesh walk kernel in the FP64 walk-for-walk mode.

* Forward mode per point and per parameter (Algorithm 2, eq. wos_deriv) on
  a displaced icosphere in a box, with one and with the 16 nested walks per
  terminal of the paper's Table 1, under the statistical parity rule of
  tests/helpers.py (3 SE + 1e-4 per comparison, at most 1% outside, mean z^2
  within 1 +- 5 sqrt(2/n)).
* Reverse mode (Sec. 5.3's weighted sum) through independent replicates.
* The ball's shape derivative du/dR against its closed form (Sec. 4):
  (sinh kr / (r sinh kR)) (1 - kR coth kR) for g = 1.
* The autograd gradient (DWoSFunction's backward) against central
  differences of the forward solve with common random numbers, and the
  eps-shell bias of the backward difference growing as eps/delta.
* Edge paths: the walk-length cap (the kmax-th query is terminal) and a
  query point with a NaN coordinate (its walks end with NaN and are counted
  as invalid, the other points' walks are unchanged).
"""
import math

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


def T(x, dev):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=dev)


def _se(v):
    return np.sqrt(np.maximum(np.asarray(v, float), 0))


def small_c3(nu=12, K=1):
    # 64 wide bumps (0.4 rad, cut at 1.2 rad): every terminal on the object
    # moves ~20 parameters, so each column of udot collects many walks
    return scenes.c3_icosphere(nu=nu, n_basis=64, h=0.4, coef_seed=0, K=K)


def shell_points(P, seed):
    # between the object (radius 0.84 .. 1.18 at nu = 12) and the box: many
    # walks end on the object
    return scenes.points_in_ball(P, 1.4, 1.85, seed)


@pytest.mark.parametrize("K", [1, 16])
def test_fp32_3d_jvp_parity_per_point_per_parameter(dev, dwos, oracle_mod, K):
    sc = small_c3(12, K)
    X = shell_points(16, 21)
    s = dwos.Solver.from_scene(sc, "fp32")
    ud, uv, um = s.jvp(T(X, dev), 4096, 301 + K)
    oud, ouv, oum, _ = oracle_mod.Oracle(sc).jvp(X, 2048, 401 + K)
    print(parity(ud.cpu().numpy(), _se(uv.cpu().numpy()), oud, _se(ouv), name=f"3D jvp K={K}"))
    # the joint u of the same walks (Sec. 5.1): it has the forward walk's
    # distribution, so a forward solve at 4096 walks gives its variance v at
    # 4096 walks per point, and 2 v at the oracle's 2048
    m, v = s.solve(T(X, dev), 4096, 501 + K)
    v = v.cpu().numpy()
    print(parity(um.cpu().numpy(), _se(v), oum, _se(2 * v), name=f"3D joint u K={K}"))


@pytest.mark.parametrize("K", [1, 16])
def test_fp32_3d_grad_parity_through_replicates(dev, dwos, oracle_mod, K):
    sc = small_c3(12, K)
    X = shell_points(16, 22)
    w = np.random.default_rng(3).normal(size=len(X))
    s = dwos.Solver.from_scene(sc, "fp32")
    R = 16
    gg = np.array([s.grad(T(X, dev), T(w, dev), 1024, 600 + r)[0].cpu().numpy() for r in range(R)])
    o = oracle_mod.Oracle(sc)
    og = np.array([o.grad(X, w, 256, 700 + r)[0] for r in range(R)])
    print(parity(gg.mean(0), gg.std(0, ddof=1) / math.sqrt(R), og.mean(0), og.std(0, ddof=1) / math.sqrt(R),
                 name=f"3D grad K={K}"))


def test_fp32_ball_shape_derivative_closed_form(dev, dwos):
    """du/dR of the ball with g = 1 and sigma = 4 (icosphere of frequency 16,
    vertices on the unit sphere): the bias budget is that of the oracle's pin
    (backward-difference offset delta = 1e-2 and the inscribed mesh), 6% of
    the largest |du/dR|."""
    sigma, k = 4.0, 2.0
    sc = scenes.sphere_scene(16, g="one", eps=1e-3, delta=1e-2, sigma=sigma)
    X = scenes.points_in_ball(16, 0.1, 0.7, 33)
    r = np.linalg.norm(X, axis=1)
    s = dwos.Solver.from_scene(sc, "fp32")
    jm, jv, _ = s.jvp(T(X, dev), 65536, 34)
    exact = np.sinh(k * r) / (r * np.sinh(k)) * (1 - k / np.tanh(k))
    print(check_vs_exact(jm.cpu().numpy()[:, 0], _se(jv.cpu().numpy()[:, 0]), exact,
                         0.06 * np.abs(exact).max(), "FP32 ball du/dR"))
    # the same through reverse mode: d/dR sum_p w_p u(x_p)
    w = np.random.default_rng(35).uniform(0.5, 1.5, len(X))
    reps = np.array([float(s.grad(T(X, dev), T(w, dev), 16384, 36 + i)[0][0]) for i in range(8)])
    ex = float(w @ exact)
    se = reps.std(ddof=1) / math.sqrt(len(reps))
    assert abs(reps.mean() - ex) <= 4 * se + 0.06 * abs(ex), (reps.mean(), ex, se)


def _wfw_records(dev, dwos, oracle_mod, sc, X, W, seed, mode):
    s = dwos.Solver.from_scene(sc, "fp64")
    g = s.walk_records(T(X, dev), W, seed, mode=mode, udot=(mode == 1))
    r = oracle_mod.Oracle(sc).walk_records(X, W, seed, mode=mode)
    return s, g, r


@pytest.mark.parametrize("mode", [0, 1])
def test_walk_for_walk_length_cap(dev, dwos, oracle_mod, mode):
    """kmax = 3: the third query of every walk that has not stopped is its
    terminal query (the walk returns g at the closest point), counted as
    truncated; FP64 GPU and oracle agree walk for walk."""
    sc = scenes.c3_icosphere(nu=4, n_basis=64, h=0.4, coef_seed=0).with_(kmax=3)
    X = shell_points(12, 23)
    s, g, r = _wfw_records(dev, dwos, oracle_mod, sc, X, 16, 24, mode)
    assert np.allclose(g["u"].cpu().numpy(), r["u"], rtol=0, atol=1e-9)
    steps = g["steps"].cpu().numpy()
    assert np.array_equal(steps, r["steps"])
    if mode == 0:
        assert steps.max() == 3
    else:
        assert np.array_equal(g["prim"].cpu().numpy(), r["prim"])
        assert np.allclose(g["uoff"].cpu().numpy(), r["uoff"], rtol=0, atol=1e-9)
        gd = g["udot"].cpu().numpy()
        assert np.allclose(gd, r["udot"], rtol=0, atol=1e-9 * max(1.0, float(np.abs(r["udot"]).max())))
    if mode == 0:
        # the library counts the walks the cap cut off, as the oracle does
        # (a forward solve runs the same walks as mode-0 records)
        m, v, st = s.solve(T(X, dev), 16, 24, stats=True)
        assert st["truncated"] == r["truncated"] > 0
        assert st["invalid"] == 0


def test_nan_point_ends_its_walks_only(dev, dwos, oracle_mod):
    """A query point with a NaN coordinate (outside any domain): its walks
    end at the first query with a NaN result and count as invalid; the
    other points (before it, so their Philox point words are unchanged)
    agree with the oracle walk for walk."""
    sc = scenes.c3_icosphere(nu=4, n_basis=64, h=0.4, coef_seed=0)
    X = shell_points(6, 25)
    Xn = np.concatenate([X, [[np.nan, 0.5, 0.5]]])
    W = 8
    s = dwos.Solver.from_scene(sc, "fp64")
    for mode in (0, 1):
        g = s.walk_records(T(Xn, dev), W, 26, mode=mode)
        r = oracle_mod.Oracle(sc).walk_records(X, W, 26, mode=mode)
        gu = g["u"].cpu().numpy()
        assert np.all(np.isnan(gu[-1]))
        assert np.allclose(gu[:-1], r["u"], rtol=0, atol=1e-9)
        assert np.array_equal(g["steps"].cpu().numpy()[:-1], r["steps"])
    m, v, st = s.solve(T(Xn, dev), W, 27, stats=True)
    assert st["invalid"] == W
    assert np.isnan(float(m[-1])) and np.all(np.isfinite(m[:-1].cpu().numpy()))
    s32 = dwos.Solver.from_scene(sc, "fp32")
    m32, _, st32 = s32.solve(T(Xn, dev), 64, 28, stats=True)
    assert st32["invalid"] == 64
    assert np.isnan(float(m32[-1])) and np.all(np.isfinite(m32[:-1].cpu().numpy()))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spatial_order_does_not_change_walks(dev, dwos, prec):
    """Calls of 1024 points or more in 3D hand their points to the walk
    kernel in a spatially coherent order; only the schedule changes: the
    first 1000 points' walks (same Philox counters) in a call of 1100 points
    equal those of a call of the 1000 points alone, bit for bit, in both
    walk kinds."""
    sc = small_c3(8)
    X = shell_points(1100, 30)
    s = dwos.Solver.from_scene(sc, prec)
    for mode in (0, 1):
        a = s.walk_records(T(X, dev), 8, 31, mode=mode, udot=(mode == 1))
        b = s.walk_records(T(X[:1000], dev), 8, 31, mode=mode, udot=(mode == 1))
        for key in ("u", "steps", "prim", "uoff") + (("udot",) if mode == 1 else ()):
            assert torch.equal(a[key][:1000], b[key]), (mode, key)
    m1, v1 = s.solve(T(X, dev), 64, 32)
    m2, v2 = s.solve(T(X[:1000], dev), 64, 32)
    assert torch.equal(m1[:1000], m2) and torch.equal(v1[:1000], v2)


def test_fp32_3d_autograd_gradient_against_central_differences(dev, dwos):
    """The autograd gradient of L(pi) = sum_p w_p u(x_p; pi) through
    DWoSFunction on the displaced icosphere (backward = differential walks,
    Algorithm 2 in reverse mode, Sec. 5.3) against central differences of the
    forward solve along three directions v, with common random numbers (the
    comparison of Sec. 6.1): both
    sides of a difference reuse the Philox stream, so a walk moves
    continuously with the boundary and the difference keeps little noise.
    Bias budget: the nested walk of the backward difference (Sec. 5.1, eq.
    dudn_fd_estimate) starts
    delta inside the boundary and stops in the eps-shell about 0.6 eps short
    of it, so the difference quotient sees an offset of about delta - 0.6 eps
    and the differential walks fall short of the eps-shell solution's
    derivative by about 0.6 eps/delta (6-7% at delta = 10 eps, measured in a
    sweep of delta down to 2.5 eps), plus the O(delta) term of the
    difference; the budget is 10% of the largest directional derivative.  The
    central difference's own O(h^2) error at h = 0.05 (surface moves below
    1e-2) lies well inside it."""
    sc = scenes.c3_icosphere(nu=12, n_basis=64, h=0.4, coef_seed=0, eps=1e-3, delta=1e-2)
    X = shell_points(32, 51)
    Xt = T(X, dev)
    w = T(np.random.default_rng(52).uniform(0.5, 1.5, len(X)), dev)
    model = dwos.ShapeModel(sc, "fp32")
    pi0 = np.asarray(sc.pi0, float)
    rng = np.random.default_rng(53)
    V = rng.normal(size=(3, sc.N))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    h, W, R = 0.05, 65536, 8

    ad = []   # g . v for each replicate (R x 3)
    for r in range(R):
        pi = torch.tensor(pi0, dtype=torch.float64, device=dev, requires_grad=True)
        u = dwos.DWoSFunction.apply(pi, Xt, model, 1024, 900 + r, W, 950 + r)
        (w * u).sum().backward()
        ad.append(V @ pi.grad.cpu().numpy())
    ad = np.array(ad)

    def L(pi, seed):
        model.apply(torch.tensor(pi, dtype=torch.float64, device=dev))
        u, _ = model.solver.solve(Xt, W, seed, var=False)
        return float((w * u).sum())

    fd = np.array([[(L(pi0 + h * v, 1000 + r) - L(pi0 - h * v, 1000 + r)) / (2 * h) for v in V]
                   for r in range(R)])
    ma, mf = ad.mean(0), fd.mean(0)
    se = np.sqrt(ad.var(0, ddof=1) / R + fd.var(0, ddof=1) / R)
    tol = 4 * se + 0.10 * np.abs(mf).max()
    print("autograd", ma, "central differences", mf, "SE", se, "tol", tol)
    assert np.abs(mf).max() > 5 * se.max(), "directional derivatives lost in noise"
    assert np.all(np.abs(ma - mf) <= tol), (ma, mf, tol)


def test_fp32_3d_eps_shell_bias_of_the_differential_walks_scales_as_eps_over_delta(dev, dwos):
    """The autograd gradient's shortfall against central differences (the
    test above) grows as delta approaches eps, as the eps-shell offset of the
    backward difference predicts: relative gap about -c eps/delta with c
    between 0.3 and 1 at delta = 10 eps and at delta = 2.5 eps, and the gap at
    2.5 eps two to six times that at 10 eps.  The gaps are pooled over three
    directions (sum of signed gaps over sum of |central difference|)."""
    eps = 1e-3
    X = shell_points(32, 51)
    Xt = T(X, dev)
    w = T(np.random.default_rng(52).uniform(0.5, 1.5, len(X)), dev)
    rng = np.random.default_rng(53)
    V = rng.normal(size=(3, 64))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    h, W, R = 0.05, 65536, 16
    fd, gaps = None, {}
    for ratio in (10.0, 2.5):
        sc = scenes.c3_icosphere(nu=12, n_basis=64, h=0.4, coef_seed=0, eps=eps, delta=ratio * eps)
        model = dwos.ShapeModel(sc, "fp32")
        pi0 = np.asarray(sc.pi0, float)
        if fd is None:   # the forward walks do not depend on delta
            def L(pi, seed):
                model.apply(torch.tensor(pi, dtype=torch.float64, device=dev))
                u, _ = model.solver.solve(Xt, W, seed, var=False)
                return float((w * u).sum())
            fd = np.array([[(L(pi0 + h * v, 1000 + r) - L(pi0 - h * v, 1000 + r)) / (2 * h) for v in V]
                           for r in range(R)])
        ad = []
        for r in range(R):
            pi = torch.tensor(pi0, dtype=torch.float64, device=dev, requires_grad=True)
            u = dwos.DWoSFunction.apply(pi, Xt, model, 1024, 900 + r, W, 950 + r)
            (w * u).sum().backward()
            ad.append(V @ pi.grad.cpu().numpy())
        ad = np.array(ad)
        s = np.sign(fd.mean(0))
        per_rep = (ad - fd) @ s / np.abs(fd.mean(0)).sum()
        gap, se = per_rep.mean(), per_rep.std(ddof=1) / math.sqrt(R)
        gaps[ratio] = gap
        print(f"delta = {ratio:g} eps: pooled relative gap {gap:.4f} (SE {se:.4f})")
        assert -1.0 / ratio - 4 * se <= gap <= -0.3 / ratio + 4 * se, (ratio, gap, se)
    assert 2.0 <= gaps[2.5] / gaps[10.0] <= 6.0, gaps
