"""The shape-optimisation step on the GPU (dwos_opt_*) against the oracle's
numpy/scipy statement of it, and the whole loop on a small 2D problem.

* The conjugate-gradient solve with M = I + lambda L equals scipy's sparse
  direct solve (icosphere, three right-hand sides).
* Several vector-Adam steps with the max second moment, with some vertices
  fixed, equal the oracle's vertex positions.
* A constant gradient translates a ring rigidly by lr per step.
* The loop (forward walks, reverse-mode differential walks with vertex
  parameters, one step, BVH refit, annealed walks per point) shrinks the
  squared loss of a 2D shape-from-diffusion problem.
"""
import numpy as np
import pytest

import scenes

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
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=dev).contiguous()


def test_cg_solve_matches_direct(dev, dwos):
    from oracle import largesteps as ls
    from scipy.sparse import linalg as spla
    V, F = scenes.icosphere(8)
    lam = 10.0
    rng = np.random.default_rng(1)
    b = rng.normal(size=(len(V), 3))
    M = ls.system_matrix(len(V), F, lam)
    ref = np.stack([spla.spsolve(M, b[:, c]) for c in range(3)], 1)
    o = dwos.LargeSteps(3, len(V), F, lam)
    x = torch.zeros(len(V), 3, dtype=torch.float64, device=dev)
    it = o.solve(T(b, dev), x, max_iters=2000, tol=1e-14)
    err = np.abs(x.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-10, (err, it)
    assert 0 < it < 2000


def test_steps_match_oracle(dev, dwos):
    from oracle import largesteps as ls
    V, F = scenes.icosphere(6)
    mv = V[:, 2] > -0.5
    lam, lr = 20.0, 0.02
    rng = np.random.default_rng(2)
    G = rng.normal(size=(5, len(V), 3))
    ref = ls.LargeSteps(V, F, lam, movable=mv, lr=lr)
    o = dwos.LargeSteps(3, len(V), F, lam, movable=mv.astype(np.int32))
    x = T(V, dev)
    o.reset(x)
    for g in G:
        xr = ref.step(g)
        o.step(T(g, dev), x, lr=lr, max_iters=3000, tol=1e-14)
        xg = x.cpu().numpy()
        assert np.abs(xg - xr).max() < 1e-9, np.abs(xg - xr).max()
        assert np.array_equal(xg[~mv], V[~mv])


def test_constant_gradient_moves_ring_rigidly(dev, dwos):
    n = 64
    th = 2 * np.pi * np.arange(n) / n
    V = np.stack([np.cos(th), np.sin(th)], 1)
    P = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    o = dwos.LargeSteps(2, n, P, 30.0)
    x = T(V, dev)
    o.reset(x)
    g = T(np.tile([[3.0, -4.0]], (n, 1)), dev)
    for k in range(3):
        o.step(g, x, lr=0.01, eps=0.0, max_iters=1000, tol=1e-14)
    assert np.allclose(x.cpu().numpy(), V + 3 * 0.01 * np.array([-0.6, 0.8]), atol=1e-10)


def test_opt_error_paths(dev, dwos):
    from paper_2405_12964_amd.capi import DwosError, DWOS_EINVAL, DWOS_ESTATE
    with pytest.raises(DwosError) as e:
        dwos.LargeSteps(4, 3, np.zeros((0, 4)), 1.0)
    assert e.value.code == DWOS_EINVAL
    with pytest.raises(DwosError) as e:
        dwos.LargeSteps(2, 3, np.array([[0, 7]]), 1.0)
    assert e.value.code == DWOS_EINVAL
    with pytest.raises(DwosError) as e:
        dwos.LargeSteps(2, 3, np.array([[0, 1]]), -1.0)
    assert e.value.code == DWOS_EINVAL
    o = dwos.LargeSteps(2, 3, np.array([[0, 1], [1, 2]]), 1.0)
    x = torch.zeros(3, 2, dtype=torch.float64, device=dev)
    with pytest.raises(DwosError) as e:
        o.step(x.clone(), x)
    assert e.value.code == DWOS_ESTATE


def _object_in_box(n, radius_fn, sigma=4.0):
    """A closed n-gon (g = 1, label 1, vertices first) inside the box
    [-2, 2]^2 (g = 0, label 0)."""
    th = 2 * np.pi * np.arange(n) / n
    r = radius_fn(th)
    Vo = np.stack([r * np.cos(th), r * np.sin(th)], 1)
    box = np.array([[-2.0, -2.0], [2.0, -2.0], [2.0, 2.0], [-2.0, 2.0]])
    V = np.concatenate([Vo, box])
    P = np.concatenate([np.stack([np.arange(n), (np.arange(n) + 1) % n], 1),
                        n + np.array([[0, 1], [1, 2], [2, 3], [3, 0]])]).astype(np.int32)
    lab = np.concatenate([np.ones(n, np.int32), np.zeros(4, np.int32)])
    return scenes.Scene(dim=2, V=V, prims=P, label=lab,
                        bc=[dict(kind="restricted", c=0.0, b=np.zeros(2), A=np.zeros((2, 2))),
                            dict(kind="restricted", c=1.0, b=np.zeros(2), A=np.zeros((2, 2)))],
                        gvert=np.zeros(len(V)), sigma=sigma, eps=1e-3, delta=1e-2)


def test_shape_from_diffusion_loop_reduces_loss(dev, dwos):
    from paper_2405_12964_amd.shapeopt import VertexShapeOptimizer
    n = 96
    target = _object_in_box(n, lambda th: 0.55 + 0.15 * np.cos(2 * th), sigma=1.0)
    start = _object_in_box(n, lambda th: 0.5 + 0 * th, sigma=1.0)
    # measurements on the inset box faces
    rng = np.random.default_rng(3)
    s_ = rng.uniform(-1.8, 1.8, 512)
    side = rng.integers(0, 4, 512)
    X = np.where(side[:, None] == 0, np.stack([s_, -1.8 + 0 * s_], 1),
        np.where(side[:, None] == 1, np.stack([1.8 + 0 * s_, s_], 1),
        np.where(side[:, None] == 2, np.stack([s_, 1.8 + 0 * s_], 1), np.stack([-1.8 + 0 * s_, s_], 1))))
    Xt = T(X, dev)
    ref = dwos.Solver.from_scene(target, "fp32")
    uref, _ = ref.solve(Xt, 4096, 7)
    mv = np.concatenate([np.ones(n, bool), np.zeros(4, bool)])
    opt = VertexShapeOptimizer(start, mv, lam=10.0, lr=1e-2, W0=32, WT=256, T=40)
    losses = []
    for t in range(40):
        L, W, its = opt.step(Xt, uref, 100 + t)
        losses.append(L)
    assert opt.t == 40 and W == 243
    assert np.mean(losses[-5:]) < 0.5 * np.mean(losses[:3]), losses
    # the fixed box did not move
    assert np.array_equal(opt.x.cpu().numpy()[n:], start.V[n:])


def test_loop_with_periodic_remeshing(dev, dwos):
    """The same loop remeshed every 10 iterations toward a finer edge length:
    the loss still falls, the box is carried over unchanged, and the object
    ends with edges within [4L/5, 4L/3] of the target."""
    from paper_2405_12964_amd.shapeopt import VertexShapeOptimizer
    n = 96
    target = _object_in_box(n, lambda th: 0.55 + 0.15 * np.cos(2 * th), sigma=1.0)
    start = _object_in_box(n, lambda th: 0.5 + 0 * th, sigma=1.0)
    rng = np.random.default_rng(3)
    s_ = rng.uniform(-1.8, 1.8, 512)
    side = rng.integers(0, 4, 512)
    X = np.where(side[:, None] == 0, np.stack([s_, -1.8 + 0 * s_], 1),
        np.where(side[:, None] == 1, np.stack([1.8 + 0 * s_, s_], 1),
        np.where(side[:, None] == 2, np.stack([s_, 1.8 + 0 * s_], 1), np.stack([-1.8 + 0 * s_, s_], 1))))
    Xt = T(X, dev)
    uref, _ = dwos.Solver.from_scene(target, "fp32").solve(Xt, 4096, 7)
    mv = np.concatenate([np.ones(n, bool), np.zeros(4, bool)])
    L = 0.8 * 2 * np.pi * 0.5 / n
    opt = VertexShapeOptimizer(start, mv, lam=10.0, lr=1e-2, W0=32, WT=256, T=40, remesh_every=10, remesh_len=L)
    losses = []
    for t in range(40):
        Lt, W, its = opt.step(Xt, uref, 100 + t)
        losses.append(Lt)
    assert np.mean(losses[-5:]) < 0.5 * np.mean(losses[:3]), losses
    V, P, mvf = opt.V, opt.P, opt.mv
    assert len(V) != n + 4                                   # the object was remeshed
    box = np.array([[-2.0, -2.0], [2.0, -2.0], [2.0, 2.0], [-2.0, 2.0]])
    assert np.array_equal(V[~mvf], box)
    seg = P[mvf[P].all(1)]
    l = np.linalg.norm(opt.x.cpu().numpy()[seg[:, 0]] - opt.x.cpu().numpy()[seg[:, 1]], axis=1)
    # edges at the last remesh were in the band; 9 optimisation steps since
    assert 0.6 * L < l.mean() < 1.5 * L
