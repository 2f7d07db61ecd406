"""Pins of the oracle's walk on stars with a Robin condition on the
reflecting boundary (Sec. 3.4, eq. (mixed_bvp): du/dn - mu u = h, n into
the domain, mu >= 0 constant, h the Robin data) and of its differential
version (Sec. 4.4, eq. (mixed_bvp_deriv): the same Robin coefficient with
zero data, nesting through the Dirichlet boundary only).

Each check is against a closed-form solution of the boundary value problem:

* the half disk with the harmonic field u = x^2 - y^2 + y: on the diameter
  du/dy = 1 and u = x^2, so Neumann data h = 1 (mu = 0) and Robin data
  h = 1 - mu x^2 both leave u exact, from points inside and from points on
  the diameter (where the walk's integral equation has u/2 on its left);
* the annulus a < r < b with u = g_a on r = a and the Robin condition on
  r = b: u = A + B ln r (Laplace) or A I0(kr) + B K0(kr) (screened), and
  its derivative in the inner radius a (a Dirichlet-boundary parameter).

Mutations that these catch: the sign of the data or Robin term, the factor
2 at wall points, the Green's function's arguments, the branch weights, the
throughput's sign.
"""
import math

import numpy as np
import pytest
from scipy import special

import scenes
from helpers import check_vs_exact


def _se(v):
    return np.sqrt(np.maximum(np.asarray(v, float), 0))


def _half_disk(mu, sigma=0.0, **kw):
    sc = scenes.half_disk_scene(g="x2-y2+y", sigma=sigma, **kw)
    return sc.with_(robin_mu=mu, robin_h=scenes._restricted(1.0, None, [[-mu, 0.0], [0.0, 0.0]], 2))


def _field(X):
    return X[:, 0] ** 2 - X[:, 1] ** 2 + X[:, 1]


@pytest.mark.parametrize("mu", [0.0, 0.7, 3.0])
def test_half_disk_robin_data_inside(oracle_mod, mu):
    """u = x^2 - y^2 + y with Robin data h = 1 - mu x^2 on the diameter (mu = 0:
    Neumann data h = 1).  Budget: the eps-shell (|grad u| eps) only."""
    sc = _half_disk(mu, eps=1e-4, delta=1e-3)
    X = scenes.points_in_half_disk(24, 71, rmax=0.9)
    m, v, _ = oracle_mod.Oracle(sc).solve(X, 8192, 72)
    check_vs_exact(m, _se(v), _field(X), 3e-4, f"half disk Robin mu={mu}")


@pytest.mark.parametrize("mu", [0.0, 1.5])
def test_half_disk_robin_data_on_the_wall(oracle_mod, mu):
    """Walks that start on the diameter: there the boundary terms carry the
    factor 2 of the wall's left side u(x)/2."""
    sc = _half_disk(mu, eps=1e-4, delta=1e-3)
    X, seg = scenes.points_on_segments(sc.NV, sc.nsegs, 16, 73)
    keep = np.abs(X[:, 0]) < 0.9
    X, seg = X[keep], seg[keep]
    m, v, _ = oracle_mod.Oracle(sc).solve(X, 8192, 74, start_seg=seg)
    check_vs_exact(m, _se(v), _field(X), 3e-4, f"half disk wall mu={mu}")


def _annulus_robin(a, b, k, mu, h, ga=1.0):
    """u = A f(r) + B h(r) with f, h = 1, ln r (k = 0) or I0(kr), K0(kr):
    u(a) = ga, -u'(b) - mu u(b) = h (the normal into the domain at r = b is
    -r/|r|)."""
    if k == 0:
        f, fp = (lambda r: np.ones_like(r)), (lambda r: np.zeros_like(r))
        g, gp = (lambda r: np.log(r)), (lambda r: 1.0 / r)
    else:
        f, fp = (lambda r: special.i0(k * r)), (lambda r: k * special.i1(k * r))
        g, gp = (lambda r: special.k0(k * r)), (lambda r: -k * special.k1(k * r))
    A = np.array([[f(np.array(a)), g(np.array(a))],
                  [-fp(np.array(b)) - mu * f(np.array(b)), -gp(np.array(b)) - mu * g(np.array(b))]], float)
    c = np.linalg.solve(A, [ga, h])
    return lambda r: c[0] * f(r) + c[1] * g(r)


def _annulus_points(n, seed, a, b):
    rng = np.random.default_rng(seed)
    r = rng.uniform(a + 0.05, b - 0.05, n)
    t = rng.uniform(0, 2 * np.pi, n)
    return np.stack([r * np.cos(t), r * np.sin(t)], 1), r


@pytest.mark.parametrize("k", [0.0, 2.0])
def test_annulus_robin_outer_wall(oracle_mod, k):
    """u = 1 on r = 0.4, du/dn - 0.8 u = 0.3 on r = 1 (polygons of 256 and 512
    sides: ~3e-5 of sagitta)."""
    a, b, mu, h = 0.4, 1.0, 0.8, 0.3
    sc = scenes.annulus_reflecting_scene(a, b, sigma=k * k).with_(
        robin_mu=mu, robin_h=scenes._restricted(h, dim=2))
    X, r = _annulus_points(24, 75, a, b)
    m, v, _ = oracle_mod.Oracle(sc).solve(X, 8192, 76)
    check_vs_exact(m, _se(v), _annulus_robin(a, b, k, mu, h)(r), 4e-4, f"annulus Robin k={k}")


def test_annulus_robin_inner_radius_derivative(oracle_mod):
    """The differential walk on stars with the Robin outer wall (Sec. 4.4:
    the derivative BVP keeps the Robin coefficient with zero data): du/da
    from the closed form's central difference in a.  Budget as the
    zero-flux pin: the backward-difference offset and the shell."""
    a, b, k, mu, h = 0.4, 1.0, 2.0, 0.8, 0.3
    sc = scenes.annulus_reflecting_scene(a, b, sigma=k * k, eps=1e-3, delta=1e-2).with_(
        robin_mu=mu, robin_h=scenes._restricted(h, dim=2))
    X, r = _annulus_points(24, 77, a, b)
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 4096, 78)
    e = 1e-6
    du = (_annulus_robin(a + e, b, k, mu, h)(r) - _annulus_robin(a - e, b, k, mu, h)(r)) / (2 * e)
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), du, 0.05 * np.abs(du).max(), "annulus Robin du/da")


def test_robin_reduces_to_zero_flux(oracle_mod):
    """mu = 0 and h = 0 given explicitly: the walks are the zero-flux walks
    plus boundary samples that change nothing (same u walk for walk, since
    the boundary sample draws from its own counters)."""
    sc0 = scenes.annulus_reflecting_scene(0.4, 1.0, sigma=4.0)
    sc1 = sc0.with_(robin_mu=0.0, robin_h=scenes._restricted(0.0, dim=2))
    X, _ = _annulus_points(6, 79, 0.4, 1.0)
    r0 = oracle_mod.Oracle(sc0).walk_records(X, 32, 80, mode=1)
    r1 = oracle_mod.Oracle(sc1).walk_records(X, 32, 80, mode=1)
    assert np.array_equal(r0["steps"], r1["steps"])
    assert np.allclose(r0["u"], r1["u"], rtol=0, atol=1e-15)
    assert np.allclose(r0["udot"], r1["udot"], rtol=0, atol=1e-15)
