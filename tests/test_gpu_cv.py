"""Learned control variate on the GPU against the FP64 oracle, through the C ABI.

* Network kernels (split-BF16 matrix-core products, FP32 accumulation) against
  the oracle's FP64 network at the same FP32 points: N, grad N, Lap N, the
  loss gradient and one Adam step.  Tolerances follow from the arithmetic: a
  split product keeps ~16 mantissa bits (relative 2^-16 = 1.5e-5 per term);
  with random-sign rounding over 64 inputs and four layers the absolute error
  of a channel stays within 1e-4 of that channel's scale (the largest
  magnitude it takes over the sample); measured: ~1.2e-5.
* Walk-for-walk (FP64 walks): run flags, alive flags, Green's-function masses,
  stop points, ball samples and the plain nested means equal the oracle's; the
  control-variate estimates differ only through the network's error.
* Statistical (FP32 walks): the differential estimate with the control
  variate agrees with the oracle's and with the closed-form shape derivative.
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


def T(x, dev, dt=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dt, device=dev)


def _scale(a):
    return float(np.max(np.abs(a))) + 1e-30


@pytest.mark.parametrize("dim", [2, 3])
def test_network_eval_matches_oracle(dev, dwos, oracle_mod, dim):
    B, th = scenes.mlp_init(dim, 31 + dim, 1.0)
    net = dwos.Network(dim, B, th)
    onet = oracle_mod.Net(dim, B.astype(np.float32).astype(np.float64),
                          th.astype(np.float32).astype(np.float64))
    rng = np.random.default_rng(dim)
    X = rng.uniform(-2, 2, (1000 + dim, dim)).astype(np.float32)   # ragged last tile
    N, G, L = net.eval(T(X, dev, torch.float32), derivatives=True)
    N0 = net.eval(T(X, dev, torch.float32))
    No, Go, Lo = onet.eval(X.astype(np.float64))
    N, G, L, N0 = (t.cpu().numpy().astype(np.float64) for t in (N, G, L, N0))
    eN, eG, eL = (np.abs(a - b).max() / _scale(b) for a, b in ((N, No), (G, Go), (L, Lo)))
    print(f"dim {dim}: rel err N {eN:.2e} grad {eG:.2e} lap {eL:.2e} (scales {_scale(No):.2f}, "
          f"{_scale(Go):.2f}, {_scale(Lo):.1f})")
    assert eN < 1e-4 and eG < 1e-4 and eL < 1e-4
    # the value-only kernel computes the same value channel
    assert np.abs(N0 - N).max() <= 1e-5 * _scale(No)


def test_network_loss_gradient_and_adam_match_oracle(dev, dwos, oracle_mod):
    dim = 3
    B, th = scenes.mlp_init(dim, 41, 1.0)
    B = B.astype(np.float32).astype(np.float64)
    th = th.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(42)
    n = 777
    X = rng.uniform(-1.5, 1.5, (n, dim)).astype(np.float32)
    Tg = rng.normal(size=n).astype(np.float32)
    w = rng.uniform(0.5, 1.5, n).astype(np.float32) / n
    net = dwos.Network(dim, B, th)
    loss, g = net.loss_grad(T(X, dev, torch.float32), T(Tg, dev, torch.float32), T(w, dev, torch.float32))
    onet = oracle_mod.Net(dim, B, th)
    Lo, go = onet.loss_grad(X.astype(np.float64), Tg.astype(np.float64), w.astype(np.float64))
    g = g.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    print(f"loss {loss.item():.6g} vs {Lo:.6g}; grad rel err {rel:.2e}")
    assert abs(loss.item() - Lo) <= 1e-4 * abs(Lo)
    assert rel < 2e-3
    # one Adam step: components whose gradient stands clear of the rounding
    # level move by exactly -lr sign(g) on both sides
    lr = 1e-3
    net.adam_step(lr)
    th1 = net.params().cpu().numpy().astype(np.float64)
    tho, m, v = th.copy(), np.zeros_like(th), np.zeros_like(th)
    oracle_mod.adam(tho, m, v, go, lr, 0.9, 0.999, 1e-8, 1)
    clear = np.abs(go) > 0.05 * np.sqrt(np.mean(go ** 2))
    assert clear.mean() > 0.3
    assert np.abs(th1 - tho)[clear].max() < 1e-6
    assert np.abs(th1 - tho).max() <= 2 * lr + 1e-6


@pytest.mark.parametrize("dim", [2, 3])
def test_network_vjp_matches_oracle(dev, dwos, oracle_mod, dim):
    """Reverse mode through the value and Laplacian channels:
    d/dtheta sum_i (Nbar_i N + Lbar_i Lap N) against the oracle (FP64)."""
    B, th = scenes.mlp_init(dim, 51 + dim, 1.0)
    B = B.astype(np.float32).astype(np.float64)
    th = th.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(52)
    n = 333
    X = rng.uniform(-1.5, 1.5, (n, dim)).astype(np.float32)
    Nb = (rng.normal(size=n) / n).astype(np.float32)
    Lb = (rng.normal(size=n) / n * 0.05).astype(np.float32)
    net = dwos.Network(dim, B, th)
    g = net.vjp(T(X, dev, torch.float32), T(Nb, dev, torch.float32), T(Lb, dev, torch.float32))
    go = oracle_mod.Net(dim, B, th).vjp(X.astype(np.float64), Nb.astype(np.float64), Lb.astype(np.float64))
    g = g.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    print(f"vjp dim {dim}: rel err {rel:.2e}")
    assert rel < 2e-3


def _disk_scene(sigma=10.0, delta=0.25, src=3.0):
    sc = scenes.c1_polygon(256, g="one", eps=1e-3, delta=delta, sigma=sigma)
    return sc.with_(src_c0=src, gauss=np.array([[5.0, 0.2, -0.1, 0.3]]))


@pytest.mark.parametrize("case", ["disk", "ball", "disk_q"])
def test_cv_walk_records_walk_for_walk(dev, dwos, oracle_mod, case):
    if case.startswith("disk"):
        sc = _disk_scene()
        X = scenes.points_in_disk(24, 0.8, 71)
    else:
        sc = scenes.sphere_scene(4, g="one", eps=4e-3, delta=0.25, sigma=4.0, source_c0=2.0)
        X = scenes.points_in_ball(12, 0.1, 0.7, 72)
    q = 0.5 if case == "disk_q" else 1.0
    B, th = scenes.mlp_init(sc.dim, 73, 1.0)
    B = B.astype(np.float32).astype(np.float64)
    th = th.astype(np.float32).astype(np.float64)
    W = 64
    ro = oracle_mod.Oracle(sc).walk_records_cv(X, W, 74, oracle_mod.Net(sc.dim, B, th, q))
    s = dwos.Solver.from_scene(sc, "fp64")
    net = dwos.Network(sc.dim, B, th)
    s.attach_cv(net, q)
    rg = {k: v.cpu().numpy() for k, v in s.cv_walk_records(T(X, dev), W, 74).items()}
    for k in ("run", "prim", "alive"):
        assert np.array_equal(rg[k], ro[k]), k
    run = ro["run"] == 1
    assert run.sum() > (0.3 if q == 1 else 0.1) * run.size
    if q < 1:
        assert (ro["run"] == 0).sum() > 0.1 * run.size
    for k in ("xoff", "uoff", "u"):
        np.testing.assert_allclose(rg[k], ro[k], rtol=1e-9, atol=1e-9, err_msg=k)
    for k in ("y", "rho", "d", "S"):
        np.testing.assert_allclose(rg[k][run], ro[k][run], rtol=1e-9, atol=1e-9, err_msg=k)
    alive = (ro["alive"] == 1) & run[..., None]
    np.testing.assert_allclose(rg["xstop"][alive], ro["xstop"][alive], rtol=1e-9, atol=1e-9)
    # the control-variate estimates: network error only.  Bound per walk:
    # |dN| (1 + 1/q) + (S |B| G / m) (|dLap| + sigma |dN|) with the network's error
    # levels eN, eL from its own parity bound (1e-4 of the channel scale)
    onet = oracle_mod.Net(sc.dim, B, th, q)
    pts = np.concatenate([ro["xoff"][..., :sc.dim].reshape(-1, sc.dim), ro["y"][..., :sc.dim].reshape(-1, sc.dim)])
    No, _, Lo = onet.eval(pts)
    eN, eL = 1e-4 * _scale(No), 1e-4 * _scale(Lo)
    Sm = ro["S"][..., 0]
    GB = np.vectorize(lambda r, R: oracle_mod.green(sc.dim, sc.sigma, r * R, R) *
                      (math.pi * R * R if sc.dim == 2 else 4 / 3 * math.pi * R ** 3) /
                      oracle_mod.green_mass(sc.dim, sc.sigma, R) if R > 0 else 0.0)(
        ro["rho"][..., 0], ro["d"][..., 0])
    bound = eN * (1 + 1 / q) + (Sm * GB * (eL + sc.sigma * eN) + eN) / q
    for k in ("uoff_cv", "target"):
        d = np.abs(rg[k] - ro[k])
        sel = ro["run"] >= 0 if k == "uoff_cv" else run
        print(f"{case} {k}: max |diff| {d[sel].max():.2e}, max bound {bound[sel].max():.2e}")
        assert np.all(d[sel] <= bound[sel] + 1e-9), k


def test_cv_fp32_gradient_parity_and_closed_form(dev, dwos, oracle_mod):
    """FP32 walks with the control variate (random network, q = 0.5): per
    point parity with the oracle's FP64 estimator and agreement with the
    closed-form du/dR of the disk, g = 1."""
    sigma = 10.0
    k = math.sqrt(sigma)
    sc = scenes.c1_polygon(256, g="one", eps=1e-3, delta=1e-2, sigma=sigma)
    X = scenes.points_in_disk(32, 0.8, 81)
    B, th = scenes.mlp_init(2, 82, 1.0)
    B = B.astype(np.float32).astype(np.float64)
    th = th.astype(np.float32).astype(np.float64)
    s = dwos.Solver.from_scene(sc, "fp32")
    net = dwos.Network(2, B, th)
    s.attach_cv(net, 0.5)
    W = 8192
    ud, uv, _ = s.jvp(T(X, dev), W, 83)
    ud, uv = ud.cpu().numpy()[:, 0], uv.cpu().numpy()[:, 0]
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 2048, 84, cv=oracle_mod.Net(2, B, th, 0.5))
    print(parity(ud, np.sqrt(uv), jm[:, 0], np.sqrt(jv[:, 0]), 1e-4, "cv jvp"))
    r = np.linalg.norm(X, axis=1)
    exact = -k * special_i0(k * r) * special_i1(k) / special_i0(k) ** 2
    check_vs_exact(ud, np.sqrt(uv), exact, 0.045 * np.abs(exact).max(), "GPU cv du/dR")


def special_i0(x):
    from scipy import special
    return special.i0(x)


def special_i1(x):
    from scipy import special
    return special.i1(x)


def test_cv_online_training_reduces_variance_and_learns_u(dev, dwos):
    """Online training (the network fitted to minimise the control variate's
    own variance on earlier walks) on the disk, g = 1, sigma = 10: the nested
    estimates' variance drops several-fold, beta approaches 1, the network
    approaches the closed form u = I0(kr)/I0(kR) at the offset points, and
    the derivative stays unbiased (closed-form du/dR)."""
    sigma = 10.0
    k = math.sqrt(sigma)
    sc = scenes.c1_polygon(512, g="one", eps=1e-3, delta=1e-2, sigma=sigma)
    X = scenes.points_in_disk(256, 0.8, 91)
    Xt = T(X, dev)
    s = dwos.Solver.from_scene(sc, "fp32")
    B, th = scenes.mlp_init(2, 4, 0.25)
    th[-(scenes.MLP_WIDTH + 1):] = 0.0
    net = dwos.Network(2, B, th)
    s.attach_cv(net, 1.0)
    for it in range(40):
        s.jvp(Xt, 256, 100 + it)
        s.cv_train(32, 8192, 1e-3, 1000 + it)
    beta = s.cv_beta()
    r = {kk: v.cpu().numpy() for kk, v in s.cv_walk_records(Xt, 256, 5000).items()}
    run = r["run"] == 1
    v_plain, v_cv = r["uoff"][run].var(), r["uoff_cv"][run].var()
    xo = r["xoff"][run][:, :2]
    No = net.eval(T(xo, dev, torch.float32)).cpu().numpy()
    uex = special_i0(k * np.linalg.norm(xo, axis=1)) / special_i0(k)
    err = np.abs(No - uex).mean()
    print(f"beta {beta:.3f} nested var {v_plain:.4g} -> {v_cv:.4g} (x{v_plain / v_cv:.1f}); "
          f"mean |N - u| at xoff {err:.2e}")
    assert beta > 0.8
    assert v_cv < v_plain / 4
    assert err < 0.01
    ud, uv, _ = s.jvp(Xt[:32], 8192, 6000)
    r32 = np.linalg.norm(X[:32], axis=1)
    exact = -k * special_i0(k * r32) * special_i1(k) / special_i0(k) ** 2
    check_vs_exact(ud.cpu().numpy()[:, 0], np.sqrt(uv.cpu().numpy()[:, 0]), exact,
                   0.045 * np.abs(exact).max(), "trained cv du/dR")
