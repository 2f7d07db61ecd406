"""The first closest-point query of each point starts from the primitive the
previous call found for that row.  Any primitive of the row's own tree only
bounds the search, so results must not depend on what the rows held: these
tests run calls whose rows hold answers for other points, other meshes or
(in a batch) other instances, and compare with a fresh context."""
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
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=dev)


def small_c3(nu, coef_seed=0):
    return scenes.c3_icosphere(nu=nu, n_basis=64, h=0.4, coef_seed=coef_seed, sigma=4.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rows_from_other_points_and_meshes(dev, dwos, prec):
    sc1, sc2 = small_c3(8), small_c3(5, coef_seed=3)
    X1 = T(scenes.points_on_box_faces(300, 1), dev)
    X2 = T(np.concatenate([scenes.points_on_box_faces(200, 2),
                           np.random.default_rng(4).uniform(-0.5, 0.5, (100, 3))]), dev)
    s = dwos.Solver.from_scene(sc1, prec)
    cold = s.walk_records(X1, 4, 11)
    again = s.walk_records(X1, 4, 11)      # warm: the rows hold these points' answers
    for k in ("u", "steps", "prim"):
        assert torch.equal(cold[k], again[k]), k
    other = s.walk_records(X2, 4, 12)      # warm from other points' answers
    fresh = dwos.Solver.from_scene(sc1, prec).walk_records(X2, 4, 12)
    for k in ("u", "steps", "prim"):
        assert torch.equal(other[k], fresh[k]), k
    # a new boundary with fewer primitives: rows are not trusted
    s.set_boundary(sc2.V, sc2.prims, sc2.label, sc2.gvert)
    got = s.walk_records(X2, 4, 13)
    ref = dwos.Solver.from_scene(sc2, prec).walk_records(X2, 4, 13)
    for k in ("u", "steps", "prim"):
        assert torch.equal(got[k], ref[k]), k


def _batch(dwos, prec, scs):
    s = dwos.Solver(3, prec)
    sc0 = scs[0]
    s.set_problem(dwos.make_problem(0.0, sc0.eps, sc0.delta, 1, sc0.kmax, 1, 0.0, None, sc0.bc, 3))
    for sc in scs:
        s.batch_add_instance(sc.V, sc.prims, sc.label, sc.sigma, sc.eps, sc.delta)
    return s


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_rows_from_other_instances(dev, dwos, prec):
    scs = [small_c3(6), small_c3(4, coef_seed=2)]
    XA = scenes.points_on_box_faces(100, 5)
    XB = scenes.points_on_box_faces(100, 6)
    s = _batch(dwos, prec, scs)
    # layout 1: 60 + 40 points; layout 2: 40 + 60, so rows 40..59 change instance
    s.batch_solve(T(np.concatenate([XA[:60], XB[:40]]), dev), [60, 40], 8, 21)
    X2 = T(np.concatenate([XA[40:80], XB[20:80]]), dev)
    m, v = s.batch_solve(X2, [40, 60], 8, 22)
    mf, vf = _batch(dwos, prec, scs).batch_solve(X2, [40, 60], 8, 22)
    assert torch.equal(m, mf) and torch.equal(v, vf)
    m2, v2 = s.batch_solve(X2, [40, 60], 8, 22)   # warm from these rows' own answers
    assert torch.equal(m, m2) and torch.equal(v, v2)
