"""The adjoint formulation of the shape derivative (Appendix B,
dwos_adjoint_grad) on the GPU against the FP64 oracle, through the C ABI.

* Walk for walk: the FP64 adjoint kernel reproduces every oracle walk (the
  adjoint estimate at the offset point, the offset mean of the K forward
  walks) within 1e-9, the gradient within 1e-9 relative and the summed step
  count exactly: the Poisson disk (one parameter), the screened star polygon
  with a Gaussian source and 16 Fourier parameters, mapped data, and the
  Poisson ball in 3D.
* FP32: the disk's finite-delta expectation (closed form, as in the oracle's
  pins) and statistical parity with the oracle on the star.
* Samples on primitives that move with no parameter run no walks.
* Error paths.
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


def T(x, dev, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device=dev)


def _ref_vec(ref, D):
    c0, b, A = ref
    b = np.zeros(D) if b is None else np.asarray(b, float)
    A = np.zeros((D, D)) if A is None else np.asarray(A, float)
    return np.concatenate([[c0], b, A.ravel()])


def _disk_poisson(delta=0.2, K=1):
    return scenes.c1_polygon(128, eps=1e-4, delta=delta, K=K).with_(bc=[scenes._restricted(0.0, dim=2)], src_c0=4.0)


def _wfw(dev, dwos, oracle_mod, sc, S, W, seed, ref):
    code, bary, wq = scenes.boundary_samples(sc, S, seed)
    s = dwos.Solver.from_scene(sc, "fp64")
    g, lam, uoff, st = s.adjoint_grad(T(code, dev, torch.int32), T(bary, dev), T(wq, dev), ref, W, seed + 1,
                                      records=True, stats=True)
    og, olam, ouoff, ost = oracle_mod.Oracle(sc).adjoint_grad(code, bary, wq, _ref_vec(ref, sc.dim), W, seed + 1)
    lam, uoff, g = lam.cpu().numpy(), uoff.cpu().numpy(), g.cpu().numpy()
    assert np.allclose(lam, olam, rtol=0, atol=1e-9), np.abs(lam - olam).max()
    assert np.allclose(uoff, ouoff, rtol=0, atol=1e-9), np.abs(uoff - ouoff).max()
    scale = max(1.0, float(np.abs(og).max()))
    assert np.allclose(g, og, rtol=0, atol=1e-9 * scale), np.abs(g - og).max()
    assert st["steps"] == int(ost.sum()), (st["steps"], int(ost.sum()))
    assert st["walks"] == S * W and st["invalid"] == 0
    return g, og


def test_walk_for_walk_disk(dev, dwos, oracle_mod):
    _wfw(dev, dwos, oracle_mod, _disk_poisson(delta=0.2, K=2), 40, 8, 11, (0.5, None, None))


def test_walk_for_walk_star_screened(dev, dwos, oracle_mod):
    sc = scenes.c2_star(256, kmax=8, coef_seed=3, sigma=4.0, eps=1e-3, delta=0.05)
    ref = (0.1, np.array([0.2, -0.1]), np.array([[0.3, 0.1], [0.0, -0.2]]))
    _wfw(dev, dwos, oracle_mod, sc, 48, 4, 12, ref)


def test_walk_for_walk_mapped(dev, dwos, oracle_mod):
    sc = scenes.c1_polygon(128, mapped=True, eps=1e-4, delta=0.1, K=2)
    _wfw(dev, dwos, oracle_mod, sc, 32, 8, 13, (0.4, None, None))


def test_walk_for_walk_ball(dev, dwos, oracle_mod):
    sc = scenes.sphere_scene(4, g="zero", eps=1e-3, delta=0.2, source_c0=6.0)
    _wfw(dev, dwos, oracle_mod, sc, 24, 4, 14, (-1.0, None, None))


def test_fp32_disk_closed_form(dev, dwos):
    """E at delta = 2 pi R [lambda(R - delta) u(R - delta) / delta^2 + c0^2/2]
    for -Lap u = 4, g = 0, uref = c0 on the unit disk."""
    R, c0, delta = 1.0, 0.5, 0.2
    sc = _disk_poisson(delta=delta)
    code, bary, wq = scenes.boundary_samples(sc, 4096, 21)
    s = dwos.Solver.from_scene(sc, "fp32")
    args = (T(code, dev, torch.int32), T(bary, dev), T(wq, dev), (c0, None, None))
    gs = [float(s.adjoint_grad(*args, 64, 100 + r)[0]) for r in range(4)]
    m, se = np.mean(gs), np.std(gs, ddof=1) / 2
    r = R - delta
    lam_x = (R * R - c0) / 4 * (R * R - r * r) - (R ** 4 - r ** 4) / 16
    exact = 2 * np.pi * R * (lam_x * (R * R - r * r) / delta ** 2 + 0.5 * c0 ** 2)
    print(f"adjoint fp32 disk: {m:.5f} +- {se:.2g} vs {exact:.5f}")
    assert abs(m - exact) <= 4.5 * se + 0.01 * exact, (m, se, exact)


def test_fp32_statistical_parity_star(dev, dwos, oracle_mod):
    sc = scenes.c2_star(256, kmax=4, coef_seed=5, sigma=4.0, eps=1e-3, delta=0.1)
    ref = (0.2, None, None)
    code, bary, wq = scenes.boundary_samples(sc, 256, 22)
    s = dwos.Solver.from_scene(sc, "fp32")
    args = (T(code, dev, torch.int32), T(bary, dev), T(wq, dev), ref)
    G = np.array([s.adjoint_grad(*args, 64, 200 + r).cpu().numpy() for r in range(8)])
    o = oracle_mod.Oracle(sc)
    O = np.array([o.adjoint_grad(code, bary, wq, _ref_vec(ref, 2), 64, 300 + r)[0] for r in range(4)])
    se = np.sqrt(G.var(0, ddof=1) / len(G) + O.var(0, ddof=1) / len(O))
    z = (G.mean(0) - O.mean(0)) / se
    print("adjoint fp32 vs oracle z-scores:", np.round(z, 2))
    assert np.all(np.abs(z) < 5.0), z


def test_fixed_primitives_run_no_walks(dev, dwos):
    """A primitive whose vertices carry no parameter adds nothing: zero
    records, no nested walks."""
    sc = _disk_poisson(delta=0.2)
    rowptr = np.zeros(sc.nv + 1, np.int64)
    rowptr[1:] = np.cumsum(np.arange(sc.nv) < 8)     # only vertices 0..7 move
    pid = np.zeros(int(rowptr[-1]), np.int32)
    vel = sc.vel[:8].copy()
    sc = sc.with_(rowptr=rowptr, pid=pid, vel=vel)
    code = np.array([100 * 2, 110 * 2], np.int32)     # primitives far from vertices 0..8
    bary = np.array([[0.3], [0.6]])
    s = dwos.Solver.from_scene(sc, "fp32")
    g, lam, uoff, st = s.adjoint_grad(T(code, dev, torch.int32), T(bary, dev), T([0.1, 0.1], dev),
                                      (0.5, None, None), 4, 1, records=True, stats=True)
    assert float(g[0]) == 0.0 and float(lam.abs().max()) == 0.0 and st["nested_walks"] == 0
    assert np.allclose(uoff.cpu().numpy(), 0.0)


def test_adjoint_error_paths(dev, dwos):
    from paper_2405_12964_amd.capi import DwosError, DWOS_EINVAL, DWOS_ESTATE
    sc = _disk_poisson()
    s = dwos.Solver.from_scene(sc, "fp32")
    code, bary, wq = scenes.boundary_samples(sc, 4, 1)
    c, b, w = T(code, dev, torch.int32), T(bary, dev), T(wq, dev)
    ref = (0.0, None, None)
    for bad in (T(code + 2 * sc.np_, dev, torch.int32), T(-np.ones(4), dev, torch.int32)):
        with pytest.raises(DwosError) as e:
            s.adjoint_grad(bad, b, w, ref, 2, 1)
        assert e.value.code == DWOS_EINVAL
    with pytest.raises(DwosError) as e:
        s.adjoint_grad(c, b, w, ref, 0, 1)
    assert e.value.code == DWOS_EINVAL
    g = s.adjoint_grad(c[:0], b[:0], w[:0], ref, 2, 1)
    assert float(g[0]) == 0.0
    # the gradient normal-derivative estimator, an implicit boundary, no parameters
    sd = dwos.Solver.from_scene(scenes.c1_polygon(64, eps=1e-3, delta=1e-2).with_(dudn=1), "fp32")
    with pytest.raises(DwosError) as e:
        sd.adjoint_grad(c, b, w, ref, 2, 1)
    assert e.value.code == DWOS_ESTATE
    sm = dwos.Solver.from_scene(scenes.monopole_scene([[0.5, 0.0, 0.0]], g=(0.0, None, None)), "fp32")
    with pytest.raises(DwosError) as e:
        sm.adjoint_grad(c, b, w, ref, 2, 1)
    assert e.value.code == DWOS_ESTATE
    sn = dwos.Solver(2, "fp32")
    sn.set_boundary(sc.V, sc.prims)
    from paper_2405_12964_amd.solver import make_problem
    sn.set_problem(make_problem(dim=2))
    with pytest.raises(DwosError) as e:
        sn.adjoint_grad(c, b, w, ref, 2, 1)
    assert e.value.code == DWOS_ESTATE
