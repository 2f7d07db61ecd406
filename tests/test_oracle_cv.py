"""Pins of the oracle's control-variate network and of the control-variate
estimator for the nested walks (CPU only).

The network and its derivative channels are pinned against central finite
differences, torch autograd (float64, CPU), special cases that reduce to
scalar library functions, and symmetries of the architecture.  The estimator
is pinned by its zero-mean identity (for a constant network it becomes an
identity of the walk itself: the killing probability equals the expected
Green's-function integral of sigma), by invariance of the mean under the
skipping probability q, and by the closed-form shape derivative of the disk.
"""
import math

import numpy as np
import pytest
import torch
from scipy import special

import scenes
from helpers import check_vs_exact

H = scenes.MLP_WIDTH


def _net(oracle_mod, dim, seed=4, q=1.0, freq=1.0):
    B, th = scenes.mlp_init(dim, seed, freq)
    return oracle_mod.Net(dim, B, th, q)


def _layer(theta, l):
    off = l * (H * H + H)
    return theta[off:off + H * H].reshape(H, H), theta[off + H * H:off + H * H + H]


def _torch_net(B, theta, dim):
    """The architecture in torch (float64) for autograd derivatives."""
    F = B.shape[0]
    Bt = torch.tensor(B)
    Ws = [(torch.tensor(_layer(theta, l)[0]), torch.tensor(_layer(theta, l)[1])) for l in range(4)]
    w5 = torch.tensor(theta[4 * (H * H + H):4 * (H * H + H) + H])
    b5 = float(theta[-1])

    def f(x):  # x: (n, dim)
        th = 2 * math.pi * x @ Bt.T
        feat = torch.cat([torch.sin(th), torch.cos(th), x,
                          torch.zeros(x.shape[0], H - 2 * F - dim, dtype=x.dtype)], dim=1)
        a = feat
        for W, b in Ws:
            a = torch.tanh(a @ W.T + b)
        return a @ w5 + b5
    return f


@pytest.mark.parametrize("dim", [2, 3])
def test_network_derivatives_match_finite_differences(oracle_mod, dim):
    net = _net(oracle_mod, dim, seed=7)
    X = np.random.default_rng(1).uniform(-1.5, 1.5, (6, dim))
    N, G, Lp = net.eval(X)
    h1 = 1e-5

    def second(x, h):   # sum of central second differences
        return sum((net.eval(x + h * e)[0][0] - 2 * net.eval(x)[0][0] + net.eval(x - h * e)[0][0])
                   / h ** 2 for e in np.eye(dim))
    for i, x in enumerate(X):
        E = np.eye(dim)
        fd_g = np.array([(net.eval(x + h1 * e)[0][0] - net.eval(x - h1 * e)[0][0]) / (2 * h1) for e in E])
        # Richardson extrapolation of the O(h^2) second differences
        fd_l = (4 * second(x, 2e-3) - second(x, 4e-3)) / 3
        np.testing.assert_allclose(G[i], fd_g, rtol=1e-6, atol=1e-6)
        assert abs(Lp[i] - fd_l) <= 1e-5 * (1 + abs(Lp[i])), (Lp[i], fd_l)


@pytest.mark.parametrize("dim", [2, 3])
def test_network_matches_torch_autograd(oracle_mod, dim):
    B, th = scenes.mlp_init(dim, 11, 1.5)
    net = oracle_mod.Net(dim, B, th)
    X = np.random.default_rng(2).uniform(-2, 2, (16, dim))
    N, G, Lp = net.eval(X)
    f = _torch_net(B, th, dim)
    x = torch.tensor(X, requires_grad=True)
    y = f(x)
    g = torch.autograd.grad(y.sum(), x, create_graph=True)[0]
    lap = sum(torch.autograd.grad(g[:, c].sum(), x, retain_graph=True)[0][:, c] for c in range(dim))
    np.testing.assert_allclose(N, y.detach().numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(G, g.detach().numpy(), rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(Lp, lap.detach().numpy(), rtol=1e-9, atol=1e-9)


def test_network_special_cases(oracle_mod):
    """Constant network; a single path through the layers reduces to a chain of
    scalar tanh/sin calls; the coordinate features enter unchanged."""
    dim, F = 3, scenes.MLP_FREQS
    B = np.random.default_rng(3).normal(size=(F, dim))
    th = np.zeros(scenes.MLP_THETA_SIZE)
    th[-1] = 0.7
    net = oracle_mod.Net(dim, B, th)
    X = np.random.default_rng(4).uniform(-1, 1, (5, dim))
    N, G, Lp = net.eval(X)
    assert np.all(N == 0.7) and np.all(G == 0) and np.all(Lp == 0)

    # path: feature -> unit 5 -> unit 9 -> unit 2 -> unit 63 -> output
    def path(feat, a, w=(0.8, -1.3, 0.6, 1.1), b=(0.1, -0.2, 0.05, 0.3), w5=2.0, b5=-0.4):
        t = np.zeros(scenes.MLP_THETA_SIZE)
        units = [5, 9, 2, 63]
        prev = feat
        for l, u in enumerate(units):
            off = l * (H * H + H)
            t[off + u * H + prev] = a if l == 0 else w[l]
            t[off + H * H + u] = b[l]
            prev = u
        t[4 * (H * H + H) + 63] = w5
        t[-1] = b5

        def ref(x, val):
            z = math.tanh(a * val + b[0])
            for l in (1, 2, 3):
                z = math.tanh(w[l] * z + b[l])
            return w5 * z + b5
        return t, ref

    for feat, fn in ((2, lambda x: math.sin(2 * math.pi * B[2] @ x)),
                     (F + 6, lambda x: math.cos(2 * math.pi * B[6] @ x)),
                     (2 * F + 1, lambda x: x[1])):
        t, ref = path(feat, 0.9)
        N, _, _ = oracle_mod.Net(dim, B, t).eval(X)
        for i, x in enumerate(X):
            assert abs(N[i] - ref(x, fn(x))) < 1e-14


def test_network_hidden_permutation_invariance(oracle_mod):
    """Relabelling the hidden units of a layer (rows of W_l, b_l and columns of
    W_{l+1}) leaves N, grad N and Lap N unchanged; a transposed weight index
    would not."""
    dim = 2
    B, th = scenes.mlp_init(dim, 5, 1.0)
    perm = np.random.default_rng(6).permutation(H)
    t2 = th.copy()
    for l in (1, 2):
        W, b = _layer(t2, l)
        Wn, _ = _layer(t2, l + 1)
        off, offn = l * (H * H + H), (l + 1) * (H * H + H)
        t2[off:off + H * H] = W[perm].ravel()
        t2[off + H * H:off + H * H + H] = b[perm]
        t2[offn:offn + H * H] = Wn[:, perm].ravel()
    X = np.random.default_rng(7).uniform(-1, 1, (8, dim))
    a = oracle_mod.Net(dim, B, th).eval(X)
    b = oracle_mod.Net(dim, B, t2).eval(X)
    for u, v in zip(a, b):
        np.testing.assert_allclose(u, v, rtol=1e-12, atol=1e-12)


def test_loss_gradient_matches_autograd_and_differences(oracle_mod):
    dim = 3
    B, th = scenes.mlp_init(dim, 8, 1.0)
    th[4 * (H * H + H) - H:4 * (H * H + H)] = np.random.default_rng(9).normal(0, 0.1, H)   # b_4
    net = oracle_mod.Net(dim, B, th)
    rng = np.random.default_rng(10)
    X = rng.uniform(-1, 1, (24, dim))
    T = rng.normal(size=24)
    w = rng.uniform(0.5, 2.0, 24)
    L, g = net.loss_grad(X, T, w)
    f = _torch_net(B, th, dim)
    # autograd with respect to theta: rebuild the net from a leaf tensor
    tt = torch.tensor(th, requires_grad=True)
    F = B.shape[0]
    xt = torch.tensor(X)
    ang = 2 * math.pi * xt @ torch.tensor(B).T
    a = torch.cat([torch.sin(ang), torch.cos(ang), xt, torch.zeros(24, H - 2 * F - dim, dtype=xt.dtype)], 1)
    for l in range(4):
        off = l * (H * H + H)
        a = torch.tanh(a @ tt[off:off + H * H].reshape(H, H).T + tt[off + H * H:off + H * H + H])
    y = a @ tt[4 * (H * H + H):4 * (H * H + H) + H] + tt[-1]
    Lt = 0.5 * (torch.tensor(w) * (y - torch.tensor(T)) ** 2).sum()
    Lt.backward()
    assert abs(L - Lt.item()) < 1e-12 * (1 + abs(L))
    np.testing.assert_allclose(g, tt.grad.numpy(), rtol=1e-9, atol=1e-12)
    # directional finite difference through the value path only
    d = rng.normal(size=th.size)
    h = 1e-6

    def loss_at(t):
        N, _, _ = oracle_mod.Net(dim, B, t).eval(X)
        return 0.5 * np.sum(w * (N - T) ** 2)
    fd = (loss_at(th + h * d) - loss_at(th - h * d)) / (2 * h)
    assert abs(fd - g @ d) < 1e-6 * (1 + abs(fd))
    del f


def test_adam_matches_torch(oracle_mod):
    rng = np.random.default_rng(12)
    n = 257
    th = rng.normal(size=n)
    m, v = np.zeros(n), np.zeros(n)
    p = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.normal(size=n) * (0.1 + step)
        oracle_mod.adam(th, m, v, g, 3e-3, 0.9, 0.999, 1e-8, step)
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def _disk(oracle_mod, sigma=10.0, src=0.0, n=256, delta=1e-2):
    sc = scenes.c1_polygon(n, g="one", eps=1e-3, delta=delta, sigma=sigma)
    if src:
        sc = sc.with_(src_c0=src)
    return sc


def test_cv_leaves_the_walks_unchanged(oracle_mod):
    """The control variate draws from its own counter purpose: the main and
    nested walks, their terminal points and plain nested means are those of
    the plain estimator; every nested walk has source steps (delta > eps), so
    its Green's-function mass S is positive."""
    sc = _disk(oracle_mod, src=3.0)
    X = scenes.points_in_disk(8, 0.8, 51)
    o = oracle_mod.Oracle(sc)
    net = _net(oracle_mod, 2, q=1.0)
    rp = o.walk_records(X, 64, 52, mode=1, want_udot=False)
    rc = o.walk_records_cv(X, 64, 52, net)
    assert np.array_equal(rp["prim"], rc["prim"])
    assert np.array_equal(rp["u"], rc["u"])
    term = rc["prim"] >= 0
    assert np.array_equal(rc["run"], np.where(term, 1, -1))
    assert np.array_equal(rp["uoff"][term], rc["uoff"][term])
    assert np.all(rc["S"][term] > 0)
    assert np.all(rc["S"][~term] == 0)
    # S is at least the mass of the selected ball
    m = np.vectorize(lambda d: oracle_mod.green_mass(2, sc.sigma, d))(rc["d"][term])
    assert np.all(rc["S"][term] >= m * (1 - 1e-12))
    # reservoir point lies in its ball; xoff is the offset of the terminal point
    dy = rc["y"][term, 0, :2] - 0  # y lies within d of the selected centre: |y| < 1
    assert np.all(np.linalg.norm(dy, axis=1) < 1.0)
    assert np.all((rc["rho"][term] > 0) & (rc["rho"][term] <= 1))
    xb = rp["xbar"][term][:, :2]
    off = np.linalg.norm(rc["xoff"][term][:, :2] - xb, axis=1)
    np.testing.assert_allclose(off, sc.delta, rtol=1e-9)
    # skipped nested walks: q = 0.3 runs about 30% of them; a skipped walk
    # uses N(xoff) alone
    net_q = _net(oracle_mod, 2, q=0.3)
    rq = o.walk_records_cv(X, 64, 52, net_q)
    run = rq["run"][term]
    assert set(np.unique(run)) <= {0, 1}
    frac = run.mean()
    assert abs(frac - 0.3) < 5 * math.sqrt(0.3 * 0.7 / run.size), frac
    Noff, _, _ = net_q.eval(rq["xoff"][term][:, :2])
    np.testing.assert_allclose(rq["uoff_cv"][term][run == 0], Noff[run == 0], rtol=1e-13)
    assert np.array_equal(rq["uoff"][term][run == 1], rp["uoff"][term][run == 1])


def _mean_se(a):
    a = np.asarray(a, float).ravel()
    return a.mean(), a.std(ddof=1) / math.sqrt(a.size)


def test_cv_constant_network_identity(oracle_mod):
    """N = 1: -Lap N + sigma N = sigma, so the zero-mean identity reads
    P(alive) + E[L |B| G sigma] = 1 -- the walk's killing probability equals its
    expected Green's-function integral of sigma.  A wrong Green's weight, a
    wrong reservoir weight or a wrong alive flag breaks it.  The nested walks start a
    quarter of the radius inside (delta = 0.25) so that they take many steps
    in large balls."""
    sc = _disk(oracle_mod, sigma=30.0, delta=0.25)
    th = np.zeros(scenes.MLP_THETA_SIZE)
    th[-1] = 1.0
    net = oracle_mod.Net(2, np.zeros((scenes.MLP_FREQS, 2)), th)
    X = scenes.points_in_disk(32, 0.8, 53)
    r = oracle_mod.Oracle(sc).walk_records_cv(X, 256, 54, net)
    term = r["run"] == 1
    C = (r["uoff_cv"] - r["uoff"])[term]
    m, se = _mean_se(C)
    assert abs(m) < 4 * se, (m, se)
    # the identity is not trivial: both terms carry weight
    assert 0.05 < r["alive"][term].mean() < 0.95


@pytest.mark.parametrize("case", ["disk_source", "ball"])
def test_cv_has_zero_mean_for_any_network(oracle_mod, case):
    """Random (untrained) network with |Lap N| ~ 100: the control variate
    changes every nested estimate but not their mean.  delta = 0.25 makes the
    nested walks long, so that the Laplacian term, the reservoir choice of
    the source step and the stop point all carry weight."""
    if case == "disk_source":
        sc = _disk(oracle_mod, sigma=10.0, src=3.0, delta=0.25)
        sc = sc.with_(gauss=np.array([[5.0, 0.2, -0.1, 0.3]]))
        X = scenes.points_in_disk(32, 0.8, 55)
        net = _net(oracle_mod, 2, seed=21, freq=1.0)
        W = 256
    else:
        sc = scenes.sphere_scene(4, g="one", eps=4e-3, delta=0.25, sigma=4.0)
        X = scenes.points_in_ball(16, 0.1, 0.7, 56)
        net = _net(oracle_mod, 3, seed=22, freq=1.0)
        W = 128
    r = oracle_mod.Oracle(sc).walk_records_cv(X, W, 57, net)
    term = r["run"] == 1
    C = (r["uoff_cv"] - r["uoff"])[term]
    m, se = _mean_se(C)
    assert abs(m) < 4 * se, (m, se)
    assert np.std(C) > 0.05     # the control variate is far from zero walk by walk


@pytest.mark.parametrize("D", [2, 3])
def test_green_mass_series(oracle_mod, D):
    """The Green's-function mass int_B G: equal to (1 - Q)/sigma where that
    has no cancellation, to the quadrature of G for tiny balls (where 1 - Q
    cancels), and to R^2/(2D) at sigma = 0."""
    from scipy import integrate
    for sigma in (0.0, 0.3, 4.0, 10.0):
        for R in (1e-4, 1e-2, 0.3, 0.9, 2.5):
            m = oracle_mod.green_mass(D, sigma, R)
            if D == 2:
                f = lambda r: oracle_mod.green(2, sigma, r, R) * 2 * math.pi * r
            else:
                f = lambda r: oracle_mod.green(3, sigma, r, R) * 4 * math.pi * r * r
            val, _ = integrate.quad(f, 0.0, R, limit=200, epsabs=0, epsrel=1e-11)
            assert m == pytest.approx(val, rel=1e-8), (D, sigma, R)
            if sigma > 0 and math.sqrt(sigma) * R > 1:
                Q = oracle_mod.poisson_scale(D, sigma, R)
                assert m == pytest.approx((1 - Q) / sigma, rel=1e-12)
            if sigma == 0:
                assert m == pytest.approx(R * R / (2 * D), rel=1e-14)


def _bowl_net(oracle_mod, dim, q=1.0):
    """A network with a definite-sign Laplacian: the sum of cos(2 pi b_i . x)
    over 16 directions b_i of length 0.15 is close to a radial paraboloid;
    one chain of tanh units on top keeps it concave and radially decreasing,
    so the Laplacian and stop-point terms have a systematic part.  The output
    bias makes N(0) = 0, which keeps the variance of the stop term small."""
    F = scenes.MLP_FREQS
    if dim == 2:
        a = 2 * np.pi * np.arange(F) / F
        dirs = np.stack([np.cos(a), np.sin(a)], 1)
    else:
        k = np.arange(F) + 0.5
        z = 1 - 2 * k / F
        ph = np.pi * (1 + 5 ** 0.5) * k
        dirs = np.stack([np.sqrt(1 - z * z) * np.cos(ph), np.sqrt(1 - z * z) * np.sin(ph), z], 1)
    B = 0.15 * dirs
    th = np.zeros(scenes.MLP_THETA_SIZE)
    th[0 * H + F:0 * H + 2 * F] = 0.1          # unit 0 of layer 1 sums the cos features
    for l in (1, 2, 3):
        th[l * (H * H + H) + 0] = 1.0           # unit 0 -> unit 0
    th[4 * (H * H + H) + 0] = 3.0
    th[-1] = -oracle_mod.Net(dim, B, th).eval(np.zeros((1, dim)))[0][0]
    return oracle_mod.Net(dim, B, th, q)


@pytest.mark.parametrize("case", ["disk_source", "ball"])
def test_cv_has_zero_mean_for_a_concave_network(oracle_mod, case):
    """With a concave, radially decreasing N the terms of the control variate
    do not average out by symmetry (Lap N < 0 everywhere, N(x_stop) < N(xoff)
    on average), so a sign error in -Lap N, a stop point taken at the wrong
    place or a source step not chosen uniformly along the walk all bias it."""
    if case == "disk_source":
        sc = _disk(oracle_mod, sigma=10.0, src=3.0, delta=0.25)
        X = scenes.points_in_disk(32, 0.8, 62)
        W = 256
    else:
        sc = scenes.sphere_scene(4, g="one", eps=4e-3, delta=0.25, sigma=4.0)
        X = scenes.points_in_ball(16, 0.1, 0.7, 63)
        W = 128
    net = _bowl_net(oracle_mod, sc.dim)
    _, _, Lp = net.eval(X)
    assert np.all(Lp < 0)
    r = oracle_mod.Oracle(sc).walk_records_cv(X, W, 64, net)
    term = r["run"] == 1
    C = (r["uoff_cv"] - r["uoff"])[term]
    m, se = _mean_se(C)
    assert abs(m) < 4 * se, (m, se)


def test_cv_has_zero_mean_for_a_residual_that_changes_along_the_walk(oracle_mod):
    """N = chain of tanh units over sum_i cos(2 pi 0.6 d_i . x) for 16
    directions d_i (close to 16 J0(3.77 r)): its residual -Lap N + sigma N is
    positive for r < 0.64 and negative beyond.  The nested walks start at
    r = 0.5 (delta = 0.5), so their first, large balls sit where the residual
    is positive and their last, small balls where it is negative: a source
    step not chosen in proportion to its ball's Green's mass (e.g. always the
    last one) biases the control variate."""
    F = scenes.MLP_FREQS
    a = 2 * np.pi * np.arange(F) / F
    B = 0.6 * np.stack([np.cos(a), np.sin(a)], 1)
    th = np.zeros(scenes.MLP_THETA_SIZE)
    th[F:2 * F] = 0.1
    for l in (1, 2, 3):
        th[l * (H * H + H)] = 1.0
    th[4 * (H * H + H)] = 10.0
    net = oracle_mod.Net(2, B, th)
    sc = _disk(oracle_mod, sigma=10.0, delta=0.5)
    P = np.array([[0.0, 0.0], [0.3, 0.2], [0.0, 0.95], [0.7, 0.68]])
    N0, _, Lp = net.eval(P)
    fN = -Lp + sc.sigma * N0
    assert fN[0] > 0 and fN[1] > 0 and fN[2] < 0 and fN[3] < 0
    X = scenes.points_in_disk(32, 0.8, 96)
    r = oracle_mod.Oracle(sc).walk_records_cv(X, 256, 97, net)
    term = r["run"] == 1
    C = (r["uoff_cv"] - r["uoff"])[term]
    m, se = _mean_se(C)
    assert abs(m) < 4 * se, (m, se)


def test_cv_mean_is_independent_of_q(oracle_mod):
    """Skipping the nested walks with probability 1 - q and reweighting the
    residual by 1/q keeps the mean: per walk the offset point is the same, so
    uoff_cv(q) - uoff(plain) has mean zero."""
    sc = _disk(oracle_mod, sigma=10.0, src=3.0)
    X = scenes.points_in_disk(32, 0.8, 58)
    o = oracle_mod.Oracle(sc)
    rp = o.walk_records(X, 256, 59, mode=1, want_udot=False)
    rq = o.walk_records_cv(X, 256, 59, _net(oracle_mod, 2, seed=23, q=0.25))
    term = rq["prim"] >= 0
    d = (rq["uoff_cv"] - rp["uoff"])[term]
    m, se = _mean_se(d)
    assert abs(m) < 4 * se, (m, se)


def test_cv_shape_derivative_disk(oracle_mod):
    """Differential WoS with the control variate (random network, q = 0.5)
    still estimates du/dR = -k I0(kr) I1(kR)/I0(kR)^2 on the disk, g = 1."""
    sigma = 10.0
    k = math.sqrt(sigma)
    sc = scenes.c1_polygon(256, g="one", eps=1e-3, delta=1e-2, sigma=sigma)
    X = scenes.points_in_disk(16, 0.8, 60)
    r = np.linalg.norm(X, axis=1)
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 2048, 61, cv=_net(oracle_mod, 2, seed=24, q=0.5))
    exact = -k * special.i0(k * r) * special.i1(k) / special.i0(k) ** 2
    check_vs_exact(jm[:, 0], np.sqrt(jv[:, 0]), exact, 0.045 * np.abs(exact).max(), "P6 disk CV")


@pytest.mark.parametrize("dim", [2, 3])
def test_value_laplacian_vjp_matches_autograd(oracle_mod, dim):
    """d/dtheta sum_i (Nbar_i N + Lbar_i Lap N) against torch's double
    backward (float64) and a directional finite difference of the oracle's
    own forward channels."""
    B, th = scenes.mlp_init(dim, 13 + dim, 1.0)
    th[np.arange(4) * (H * H + H) + H * H] = 0.1   # some nonzero biases
    net = oracle_mod.Net(dim, B, th)
    rng = np.random.default_rng(20 + dim)
    n = 9
    X = rng.uniform(-1.2, 1.2, (n, dim))
    Nb, Lb = rng.normal(size=n), rng.normal(size=n) * 0.1
    g = net.vjp(X, Nb, Lb)
    # autograd: rebuild the network from a leaf theta
    tt = torch.tensor(th, requires_grad=True)
    F = B.shape[0]
    x = torch.tensor(X, requires_grad=True)
    ang = 2 * math.pi * x @ torch.tensor(B).T
    a = torch.cat([torch.sin(ang), torch.cos(ang), x, torch.zeros(n, H - 2 * F - dim, dtype=x.dtype)], 1)
    for l in range(4):
        off = l * (H * H + H)
        a = torch.tanh(a @ tt[off:off + H * H].reshape(H, H).T + tt[off + H * H:off + H * H + H])
    y = a @ tt[4 * (H * H + H):4 * (H * H + H) + H] + tt[-1]
    gx = torch.autograd.grad(y.sum(), x, create_graph=True)[0]
    lap = sum(torch.autograd.grad(gx[:, c].sum(), x, create_graph=True)[0][:, c] for c in range(dim))
    obj = (torch.tensor(Nb) * y).sum() + (torch.tensor(Lb) * lap).sum()
    gt = torch.autograd.grad(obj, tt)[0].numpy()
    np.testing.assert_allclose(g, gt, rtol=1e-8, atol=1e-10)
    d = rng.normal(size=th.size)
    h = 1e-6

    def f(t):
        N, _, L = oracle_mod.Net(dim, B, t).eval(X)
        return float(Nb @ N + Lb @ L)
    fd = (f(th + h * d) - f(th - h * d)) / (2 * h)
    assert abs(fd - g @ d) < 1e-5 * (1 + abs(fd))
