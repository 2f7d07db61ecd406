"""Reverse mode over a batch of instances in one launch (dwos_batch_grad).

* FP64 (instances share the boundary-data table, as a batch context does):
  each instance's slice of the batch gradient, and the joint u
  estimates, equal the oracle's reverse mode for that instance with its
  instance index in the Philox counter (same walks), within 1e-9.
* FP32: two screened disks of different radius and screening, g = 1, each
  with its radius as parameter: each slice against the closed form
  mean_p du/dR = -mean_p I0(k r_p) k I1(k R) / I0(k R)^2.
* Error paths: instances with different delta, no parameters, single-problem
  calls on a batch context.
"""
import numpy as np
import pytest
from scipy import special

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
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=dev)


def _batch(dwos, prec, scs):
    from paper_2405_12964_amd.solver import make_problem
    s = dwos.Solver(2, prec)
    s0 = scs[0]
    s.set_problem(make_problem(0.0, s0.eps, s0.delta, s0.K, s0.kmax, s0.rr, s0.src_c0, s0.gauss, s0.bc, 2))
    for i, sc in enumerate(scs):
        idx = s.batch_add_instance(sc.V, sc.prims, sc.label, sc.sigma, sc.eps, sc.delta)
        assert idx == i
        s.batch_set_parameters(i, sc.N, sc.rowptr, sc.pid, sc.vel)
    return s


def test_batch_grad_equals_oracle_per_instance(dev, dwos, oracle_mod):
    scs = [scenes.c1_polygon(64, R=1.0, g="one", eps=1e-3, delta=1e-2, sigma=4.0),
           scenes.c1_polygon(96, R=0.8, g="one", eps=2e-3, delta=1e-2, sigma=9.0),
           scenes.c1_polygon(48, R=1.2, g="one", eps=1e-3, delta=1e-2, sigma=0.5)]
    P = [5, 7, 3]
    Xs = [scenes.points_in_disk(p, 0.7 * sc.pi0[0], 40 + i) for i, (p, sc) in enumerate(zip(P, scs))]
    rng = np.random.default_rng(3)
    ws = [rng.normal(size=p) for p in P]
    W, seed = 16, 77
    s = _batch(dwos, "fp64", scs)
    g, um = s.batch_grad(T(np.concatenate(Xs), dev), P, T(np.concatenate(ws), dev), W, seed)
    g, um = g.cpu().numpy(), um.cpu().numpy()
    off = 0
    for i, sc in enumerate(scs):
        og, oum, _ = oracle_mod.Oracle(sc).grad(Xs[i], ws[i], W, seed, instance=i)
        assert np.allclose(g[i:i + 1], og, rtol=0, atol=1e-9 * max(1.0, np.abs(og).max())), (i, g[i], og)
        assert np.allclose(um[off:off + P[i]], oum, rtol=0, atol=1e-9)
        off += P[i]


def test_batch_grad_closed_form_fp32(dev, dwos):
    scs = [scenes.c1_polygon(512, R=1.0, g="one", eps=1e-3, delta=1e-2, sigma=10.0),
           scenes.c1_polygon(512, R=0.7, g="one", eps=1e-3, delta=1e-2, sigma=4.0)]
    P = [256, 256]
    Xs = [scenes.points_in_disk(p, 0.8 * sc.pi0[0], 50 + i) for i, (p, sc) in enumerate(zip(P, scs))]
    ws = [np.full(p, 1.0 / p) for p in P]
    s = _batch(dwos, "fp32", scs)
    g, _ = s.batch_grad(T(np.concatenate(Xs), dev), P, T(np.concatenate(ws), dev), 4096, 5)
    g = g.cpu().numpy()
    for i, sc in enumerate(scs):
        k, R = np.sqrt(sc.sigma), sc.pi0[0]
        r = np.linalg.norm(Xs[i], axis=1)
        exact = np.mean(-special.i0(k * r) * k * special.i1(k * R) / special.i0(k * R) ** 2)
        # bias budget of the backward difference (delta/2 u_rr, ~4%) and the polygon
        assert abs(g[i] - exact) < 0.06 * abs(exact), (i, g[i], exact)


def test_batch_grad_error_paths(dev, dwos):
    from paper_2405_12964_amd.capi import DwosError, DWOS_EINVAL, DWOS_ESTATE
    a = scenes.c1_polygon(32, g="one", eps=1e-3, delta=1e-2, sigma=1.0)
    b = scenes.c1_polygon(32, g="one", eps=1e-3, delta=2e-2, sigma=1.0)
    X = T(np.concatenate([scenes.points_in_disk(2, 0.5, 1), scenes.points_in_disk(2, 0.5, 2)]), dev)
    w = T(np.ones(4), dev)
    s = _batch(dwos, "fp32", [a, b])
    with pytest.raises(DwosError) as e:
        s.batch_grad(X, [2, 2], w, 4, 1)
    assert e.value.code == DWOS_EINVAL
    s = _batch(dwos, "fp32", [a, a])
    s.batch_set_parameters(0, 0)
    s.batch_set_parameters(1, 0)
    with pytest.raises(DwosError) as e:
        s.batch_grad(X, [2, 2], w, 4, 1)
    assert e.value.code == DWOS_ESTATE
    with pytest.raises(DwosError) as e:
        s.batch_set_parameters(5, 1, a.rowptr, a.pid, a.vel)
    assert e.value.code == DWOS_EINVAL
    # single-problem calls on a batch context
    for call in (lambda: s.solve(X, 4, 1), lambda: s.grad(X, w, 4, 1), lambda: s.closest(X)):
        with pytest.raises(DwosError) as e:
            call()
        assert e.value.code == DWOS_ESTATE


def test_batch_screened_instance_needs_roulette(dev, dwos):
    """An instance with sigma > 0 in a batch whose problem has roulette off
    (rr = 0) is rejected by both batch calls: without roulette the walks would
    drop the attenuation factors of the screened walk (Sec. 3.3)."""
    from paper_2405_12964_amd.capi import DwosError, DWOS_EINVAL
    from paper_2405_12964_amd.solver import make_problem
    a = scenes.c1_polygon(32, g="one", eps=1e-3, delta=1e-2, sigma=0.0)
    b = scenes.c1_polygon(32, g="one", eps=1e-3, delta=1e-2, sigma=3.0)
    X = T(np.concatenate([scenes.points_in_disk(2, 0.5, 1), scenes.points_in_disk(2, 0.5, 2)]), dev)
    w = T(np.ones(4), dev)
    s = dwos.Solver(2, "fp32")
    s.set_problem(make_problem(0.0, a.eps, a.delta, 1, a.kmax, 0, 0.0, None, a.bc, 2))
    for sc in (a, b):
        i = s.batch_add_instance(sc.V, sc.prims, sc.label, sc.sigma, sc.eps, sc.delta)
        s.batch_set_parameters(i, sc.N, sc.rowptr, sc.pid, sc.vel)
    for call in (lambda: s.batch_solve(X, [2, 2], 4, 1), lambda: s.batch_grad(X, [2, 2], w, 4, 1)):
        with pytest.raises(DwosError) as e:
            call()
        assert e.value.code == DWOS_EINVAL
    # with roulette on, the same batch runs
    s.set_problem(make_problem(0.0, a.eps, a.delta, 1, a.kmax, 1, 0.0, None, a.bc, 2))
    m, _ = s.batch_solve(X, [2, 2], 16, 1)
    assert np.all(np.isfinite(m.cpu().numpy()))


def _batch3d(dwos, insts, stream=None):
    from paper_2405_12964_amd.solver import make_problem
    s = dwos.Solver(3, "fp32", stream=stream)
    sc0 = insts[0][0]
    s.set_problem(make_problem(0.0, sc0.eps, sc0.delta, 1, sc0.kmax, 1, 0.0, None, sc0.bc, 3))
    for i, (sc, _) in enumerate(insts):
        assert s.batch_add_instance(sc.V, sc.prims, sc.label, sc.sigma, sc.eps, sc.delta) == i
        s.batch_set_parameters(i, sc.N, sc.rowptr, sc.pid, sc.vel)
    return s


def test_batch_graph_capture_replays_match_eager(dev, dwos):
    """Batched instances of the 3D generator of the batch workload (displaced
    icospheres in boxes, uneven sizes, screening sigma ~ U(0, 20)): the
    batched solve and reverse mode captured in one hipGraph on the context
    stream and replayed with a new device seed each time equal the eager calls
    with that seed (the gradient to the FP64 atomics' summation order), with
    eager work between replays."""
    insts = scenes.c4_batch(n_inst=6, tri_lo=200, tri_hi=3000, p_lo=32, p_hi=256, n_basis=16)
    X = T(np.concatenate([x for _, x in insts]), dev)
    P = [len(x) for _, x in insts]
    w = torch.linspace(-1, 1, X.shape[0], dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = _batch3d(dwos, insts, stream)
        seed_buf = torch.zeros(1, dtype=torch.int64, device=dev)
        s.set_seed_buffer(seed_buf)
        s.batch_solve(X, P, 64, 5)
        s.batch_grad(X, P, w, 64, 6)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        mg, vg = s.batch_solve(X, P, 64, 5)
        gg, ug = s.batch_grad(X, P, w, 64, 6)
    outs = []
    for r in range(4):
        with torch.cuda.stream(stream):
            seed_buf.fill_(2000 + r)
            g.replay()
            me, ve = s.batch_solve(X, P, 64, 5)
            ge, ue = s.batch_grad(X, P, w, 64, 6)
        torch.cuda.synchronize()
        assert torch.equal(mg, me) and torch.equal(vg, ve), r
        assert torch.allclose(gg, ge, rtol=1e-12, atol=1e-14) and torch.equal(ug, ue), r
        outs.append(mg.clone())
        _ = torch.randn(1000, device=dev).sum().item()
    assert not torch.equal(outs[0], outs[1])
    s.set_seed_buffer(None)


def test_batch_grad_3d_equals_oracle_per_instance(dev, dwos, oracle_mod):
    """3D instances of the batch generator (FP64 walk for walk): each
    instance's slice of the batch gradient equals the oracle's reverse mode of
    that instance with its instance index in the Philox counter."""
    insts = scenes.c4_batch(n_inst=3, tri_lo=150, tri_hi=800, p_lo=6, p_hi=10, n_basis=16)
    from paper_2405_12964_amd.solver import make_problem
    s = dwos.Solver(3, "fp64")
    sc0 = insts[0][0]
    s.set_problem(make_problem(0.0, sc0.eps, sc0.delta, 1, sc0.kmax, 1, 0.0, None, sc0.bc, 3))
    for i, (sc, _) in enumerate(insts):
        s.batch_add_instance(sc.V, sc.prims, sc.label, sc.sigma, sc.eps, sc.delta)
        s.batch_set_parameters(i, sc.N, sc.rowptr, sc.pid, sc.vel)
    X = np.concatenate([x for _, x in insts])
    P = [len(x) for _, x in insts]
    rng = np.random.default_rng(7)
    w = rng.normal(size=len(X))
    W, seed = 16, 31
    g, um = s.batch_grad(T(X, dev), P, T(w, dev), W, seed)
    g = g.cpu().numpy()
    off, p0 = 0, 0
    for i, (sc, x) in enumerate(insts):
        og, oum, _ = oracle_mod.Oracle(sc).grad(x, w[p0:p0 + len(x)], W, seed, instance=i)
        gi = g[off:off + sc.N]
        assert np.allclose(gi, og, rtol=1e-9, atol=1e-9 * max(1.0, float(np.abs(og).max()))), (i, gi, og)
        assert np.allclose(um.cpu().numpy()[p0:p0 + len(x)], oum, rtol=0, atol=1e-9), i
        off += sc.N
        p0 += len(x)
