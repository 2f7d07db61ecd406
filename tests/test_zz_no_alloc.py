"""The allocation-free solve (dwos_solve_noalloc) against dwos_solve.

Both run the same walks from the same Philox streams with the same kernels,
so their per-point means and variances agree exactly; checked on two calls in
a row (the second smaller, so stale workspace contents from the first would
show), in FP32 and FP64, 2D and 3D, plus the size limit and error paths.
"""
import ctypes as C

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


def T(x, dev):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=dev)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("which", ["star", "c3"])
def test_noalloc_equals_solve_on_two_calls(dev, prec, which):
    from paper_2405_12964_amd import Solver
    if which == "star":
        sc = scenes.c2_star(n=1024, kmax=8)
        X1, X2 = scenes.star_points(3000, 1), scenes.star_points(700, 2)
        W1, W2 = 512, 96
    else:
        sc = scenes.c3_icosphere(nu=20, n_basis=64, h=0.4, coef_seed=0)
        X1, X2 = scenes.points_on_box_faces(2048, 1), scenes.points_on_box_faces(333, 2)
        W1, W2 = 256, 40
    s = Solver.from_scene(sc, prec)
    for X, W, seed in ((X1, W1, 11), (X2, W2, 12)):
        Xt = T(X, dev)
        m_ref, v_ref = s.solve(Xt, W, seed)
        m = torch.full((len(X),), np.nan, dtype=torch.float64, device=dev)
        v = torch.full((len(X),), np.nan, dtype=torch.float64, device=dev)
        s.solve_noalloc(Xt, W, seed, m, v)
        torch.cuda.synchronize()
        assert torch.equal(m, m_ref), float((m - m_ref).abs().max())
        assert torch.equal(v, v_ref), float((v - v_ref).abs().max())
        # without the variance output
        m2 = torch.full((len(X),), np.nan, dtype=torch.float64, device=dev)
        s.solve_noalloc(Xt, W, seed, m2, None)
        torch.cuda.synchronize()
        assert torch.equal(m2, m_ref)


def test_noalloc_limits_and_errors(dev):
    from paper_2405_12964_amd import Solver, capi
    from paper_2405_12964_amd.capi import DwosError
    sc = scenes.c2_star(n=256)
    s = Solver.from_scene(sc, "fp32")
    X = T(scenes.star_points(64, 3), dev)
    m = torch.empty(64, dtype=torch.float64, device=dev)
    # 64 points x 2^18 walks need 64 MiB of FP32 walk values: beyond the 32 MiB array
    with pytest.raises(DwosError) as e:
        s.solve_noalloc(X, 1 << 18, 1, m)
    assert e.value.code == capi.DWOS_EINVAL
    with pytest.raises(DwosError) as e:
        s.solve_noalloc(X, 0, 1, m)
    assert e.value.code == capi.DWOS_EINVAL
    assert capi.dwos_solve_noalloc(None, None, 0, 1, 0, None, None) == capi.DWOS_EINVAL
    # an empty call is accepted and touches nothing
    assert capi.dwos_solve_noalloc(s._ctx, None, 0, 8, 0, None, None) == capi.DWOS_OK
    # the largest FP32 solve that fits still agrees with dwos_solve
    P, W = 64, 120000
    mr, vr = s.solve(X, W, 5)
    m2 = torch.empty(P, dtype=torch.float64, device=dev)
    v2 = torch.empty(P, dtype=torch.float64, device=dev)
    s.solve_noalloc(X, W, 5, m2, v2)
    torch.cuda.synchronize()
    assert torch.equal(m2, mr) and torch.equal(v2, vr)
