"""Pins of the oracle's walk on stars (mixed Dirichlet / zero-flux problems,
Sec. 3.4 eq. (mixed_bvp); differential version Sec. 4.4, eq. (mixed_bvp_deriv)).

The reflecting-boundary machinery is checked against things fixed outside
the oracle:

* the step weight against the ball's Green's function (finite differences of
  G, and an independent Bessel library);
* silhouette distances and ray hits against the geometry of the L-shaped
  domain worked out by hand, and star-shapedness against brute-force
  visibility sampling;
* whole walks against closed-form solutions: the re-entrant corner
  r^(2/3) cos(2 theta/3) (Laplace) and I_{2/3}(k r) cos(2 theta/3)
  (screened), mirror symmetry on the half disk, the annulus with a reflecting
  outer wall and its derivative in the inner radius, the half disk's
  derivative in its radius, and walks that start on the reflecting wall;
* the exact reduction to Algorithm 1 when the reflecting boundary is out of
  reach (the walks then coincide step for step).
"""
import math

import numpy as np
import pytest
from scipy import special

import scenes
from helpers import check_vs_exact


def _se(v):
    return np.sqrt(np.maximum(np.asarray(v, float), 0))


def _polar(X):
    r = np.hypot(X[:, 0], X[:, 1])
    th = np.mod(np.arctan2(X[:, 1], X[:, 0]), 2 * np.pi)
    return r, th


# ----------------------------------------------------------- step weight ----

@pytest.mark.parametrize("sigma", [0.5, 4.0, 40.0])
@pytest.mark.parametrize("dim", [2, 3])
def test_neumann_weight_is_green_derivative(oracle_mod, sigma, dim):
    """w(r; R) = |dS_1| r^(D-1) |dG/dr| (central differences of G), equals
    alpha(R) at r = R and tends to 1 as r -> 0."""
    area = 2 * math.pi if dim == 2 else 4 * math.pi
    for R in (0.05, 0.4, 1.3):
        for f in (0.01, 0.2, 0.5, 0.9, 0.99):
            r = f * R
            h = 1e-6 * r
            dG = (oracle_mod.green(dim, sigma, r + h, R) - oracle_mod.green(dim, sigma, r - h, R)) / (2 * h)
            ref = area * r ** (dim - 1) * abs(dG)
            w = oracle_mod.neumann_weight(dim, sigma, r, R)
            assert abs(w - ref) <= 1e-6 * ref, (dim, sigma, R, r, w, ref)
        assert abs(oracle_mod.neumann_weight(dim, sigma, R, R) - oracle_mod.poisson_scale(dim, sigma, R)) < 1e-12
        assert abs(oracle_mod.neumann_weight(dim, sigma, 1e-9 * R, R) - 1) < 1e-6
    assert oracle_mod.neumann_weight(dim, 0.0, 0.3, 1.0) == 1.0


def test_neumann_weight_vs_scipy(oracle_mod):
    """2D: k r [K1(kr) + K0(kR) I1(kr)/I0(kR)] with scipy's Bessel functions."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        k, R = rng.uniform(0.1, 8.0), rng.uniform(0.01, 2.0)
        r = rng.uniform(0.001, 1.0) * R
        a, b = k * r, k * R
        ref = a * (special.k1(a) + special.k0(b) * special.i1(a) / special.i0(b))
        assert abs(oracle_mod.neumann_weight(2, k * k, r, R) - ref) <= 1e-12 * ref


# ------------------------------------------------- silhouettes and rays ----

@pytest.fixture(scope="module")
def lshape(oracle_mod):
    sc = scenes.lshape_scene()
    return sc, oracle_mod.Oracle(sc)


def _lshape_silhouette(x):
    """By hand: the re-entrant corner (origin) is a silhouette unless x is in
    the quadrant x < 0, y > 0 (from there both walls face x); the open ends
    (1, 0) and (0, -1) always are; the collinear wall vertices never are."""
    c = [np.hypot(x[0] - 1, x[1]), np.hypot(x[0], x[1] + 1)]
    if not (x[0] < 0 and x[1] > 0):
        c.append(np.hypot(x[0], x[1]))
    return min(c)


def test_silhouette_distance_lshape(lshape):
    sc, o = lshape
    X = scenes.points_in_lshape(400, 5)
    for x in X:
        assert abs(o.silhouette(x) - _lshape_silhouette(x)) < 1e-12, x


def test_silhouette_on_the_wall(lshape):
    """x on a wall (domain side given): the corner is a silhouette (the other
    wall leaves to the outside of this wall's line), the wall's own vertices
    are not, so the distance is the distance to the corner (or to the open
    end, if nearer)."""
    sc, o = lshape
    for s in (0.05, 0.3, 0.7):
        d = o.silhouette([s, 0.0], on=16 + int(s * 16), nin=[0.0, 1.0])
        assert abs(d - min(s, 1 - s)) < 1e-12
        d = o.silhouette([0.0, -s], on=15 - int(s * 16), nin=[-1.0, 0.0])
        assert abs(d - min(s, 1 - s)) < 1e-12
    # a point on the wall next to the corner, rounded a hair off the wall's
    # line to the outside: the corner still counts (the wall it lies on is
    # edge-on by construction, not by the sign of a rounded cross product)
    for off in (1e-9, -1e-9):
        assert abs(o.silhouette([0.03, off], on=16, nin=[0.0, 1.0]) - np.hypot(0.03, off)) < 1e-12
        assert abs(o.silhouette([off, -0.03], on=15, nin=[-1.0, 0.0]) - np.hypot(0.03, off)) < 1e-12


def test_silhouette_on_a_straight_subdivided_wall(oracle_mod):
    """Half disk: from a point on the (64-segment) diameter, the only
    silhouettes are the open ends; without the on-wall rule every wall vertex
    would be counted (x is collinear with all of them)."""
    sc = scenes.half_disk_scene()
    o = oracle_mod.Oracle(sc)
    for xs in (-0.8, -0.31, 0.0, 0.52):
        seg = int((xs + 1) / (2 / 64))
        assert abs(o.silhouette([xs, 0.0], on=seg, nin=[0, 1]) - (1 - abs(xs))) < 1e-12
    # inside a convex domain: only the open ends
    for x in scenes.points_in_half_disk(50, 3):
        ends = min(np.hypot(x[0] - 1, x[1]), np.hypot(x[0] + 1, x[1]))
        assert abs(o.silhouette(x) - ends) < 1e-12


def _visible(x, y):
    """Does the segment x-y stay in the L-shaped domain (no wall crossing)?"""
    t = np.linspace(0, 1, 400)[1:]
    P = x[None, :] + t[:, None] * (y - x)[None, :]
    return not np.any((P[:, 0] > 0) & (P[:, 1] < 0))


def test_star_radius_is_star_shaped_and_tight(lshape):
    """Brute-force visibility: every domain point within the star radius
    min(d_Dirichlet, d_silhouette) is visible from x; and where the corner is
    the binding silhouette, some point just beyond it is not."""
    sc, o = lshape
    rng = np.random.default_rng(9)
    X = scenes.points_in_lshape(60, 11)
    tight = 0
    for x in X:
        dD = o.closest(x)["d"]
        R = min(dD, o.silhouette(x))
        Y = x + R * np.sqrt(rng.random((300, 1))) * _dirs(rng, 300)
        Y = Y[~((Y[:, 0] > 0) & (Y[:, 1] < 0))]
        assert all(_visible(x, y) for y in Y), x
        if abs(R - np.hypot(*x)) < 1e-12 and R < dD - 0.05:
            # a point behind the corner at distance 1.02 R is hidden
            u = -x / np.hypot(*x)
            far = x + 1.02 * R * (u + np.array([u[1], -u[0]]) * 0.1 * np.sign(x[0] - x[1]))
            if not ((far[0] > 0) and (far[1] < 0)):
                tight += not _visible(x, far)
    assert tight > 0


def _dirs(rng, n):
    a = 2 * np.pi * rng.random(n)
    return np.stack([np.cos(a), np.sin(a)], 1)


def test_ray_hits_lshape(lshape):
    """Rays against the walls y = 0 (x in [0, 1]) and x = 0 (y in [-1, 0])."""
    sc, o = lshape
    rng = np.random.default_rng(12)
    for x in scenes.points_in_lshape(200, 13):
        d = _dirs(rng, 1)[0]
        hits = []
        if d[1] != 0:
            t = -x[1] / d[1]
            if t > 0 and 0 <= x[0] + t * d[0] <= 1:
                hits.append(t)
        if d[0] != 0:
            t = -x[0] / d[0]
            if t > 0 and -1 <= x[1] + t * d[1] <= 0:
                hits.append(t)
        t, seg = o.ray(x, d, 10.0)
        if hits:
            assert abs(t - min(hits)) < 1e-12 and seg >= 0
        else:
            assert seg == -1 and t == 10.0
        t2, seg2 = o.ray(x, d, 0.5 * t if seg >= 0 else 10.0)
        assert seg2 == -1


# -------------------------------------------------------- closed forms -----

def test_reentrant_corner_laplace(lshape):
    """-Lap u = 0 in the L-shape, zero flux on both walls of the re-entrant
    corner: u = r^(2/3) cos(2 theta/3).  Bias: shell (|grad u| eps ~ 1e-4)
    and the piecewise-linear data (h^2/8 |g''| ~ 4e-6)."""
    sc, o = lshape
    X = scenes.points_in_lshape(24, 21)
    m, v, _ = o.solve(X, 8192, 22)
    r, th = _polar(X)
    check_vs_exact(m, _se(v), scenes.corner_harmonic(r, th), 3e-4, "L-shape Laplace")


def test_reentrant_corner_screened(oracle_mod):
    """-Lap u + k^2 u = 0: u = I_{2/3}(k r) cos(2 theta/3); exercises the
    Bessel weights of steps ending on a wall."""
    k = 2.0
    g = lambda r, th: special.iv(2.0 / 3.0, k * r) * np.cos(2 * th / 3)
    sc = scenes.lshape_scene(sigma=k * k, gfun=g)
    X = scenes.points_in_lshape(24, 23)
    m, v, _ = oracle_mod.Oracle(sc).solve(X, 8192, 24)
    r, th = _polar(X)
    check_vs_exact(m, _se(v), g(r, th), 3e-4, "L-shape screened")


def test_wall_orientation_does_not_matter_inside(oracle_mod):
    """The walls' segment direction only names the domain side of a start
    point; a walk that reaches a wall takes the side it came from.  With
    every wall reversed the interior solution is unchanged."""
    sc = scenes.lshape_scene()
    sc = sc.with_(nsegs=np.ascontiguousarray(sc.nsegs[:, ::-1]))
    X = scenes.points_in_lshape(24, 21)
    m, v, _ = oracle_mod.Oracle(sc).solve(X, 8192, 27)
    r, th = _polar(X)
    check_vs_exact(m, _se(v), scenes.corner_harmonic(r, th), 3e-4, "L-shape reversed walls")


def test_walks_starting_on_the_wall(lshape, oracle_mod):
    """Points on the walls: u = r^(2/3) on theta = 0 and -r^(2/3) on
    theta = 3 pi / 2 (hemisphere sampling at the start)."""
    sc, o = lshape
    X, seg = scenes.points_on_segments(sc.NV, sc.nsegs, 24, 25)
    m, v, _ = o.solve(X, 8192, 26, start_seg=seg)
    r, th = _polar(X)
    check_vs_exact(m, _se(v), scenes.corner_harmonic(r, th), 3e-4, "L-shape on wall")


def test_half_disk_mirror(oracle_mod):
    """Half disk with a reflecting diameter: data even in y give the full
    disk's solution, x^2 - y^2 (Laplace) and I0(kr)/I0(k) (screened);
    also from points on the diameter."""
    X = scenes.points_in_half_disk(24, 27)
    sc = scenes.half_disk_scene()
    o = oracle_mod.Oracle(sc)
    m, v, _ = o.solve(X, 8192, 28)
    check_vs_exact(m, _se(v), X[:, 0] ** 2 - X[:, 1] ** 2, 3e-4, "half disk x2-y2")
    Xw, seg = scenes.points_on_segments(sc.NV, sc.nsegs, 16, 29)
    m, v, _ = o.solve(Xw, 8192, 30, start_seg=seg)
    check_vs_exact(m, _se(v), Xw[:, 0] ** 2, 3e-4, "half disk x2-y2 on wall")
    k = 3.0
    o = oracle_mod.Oracle(scenes.half_disk_scene(sigma=k * k, g="one"))
    m, v, _ = o.solve(X, 8192, 31)
    r = np.hypot(X[:, 0], X[:, 1])
    check_vs_exact(m, _se(v), special.i0(k * r) / special.i0(k), 5e-4, "half disk screened")


def test_half_disk_source(oracle_mod):
    """Constant source f with u = 0 on the arc: the source sample of a step
    counts only inside the star-shaped region (rho < t).  Laplace:
    u = f (1 - r^2)/4; screened: u = (f/k^2)(1 - I0(kr)/I0(k))."""
    X = scenes.points_in_half_disk(24, 41)
    r = np.hypot(X[:, 0], X[:, 1])
    o = oracle_mod.Oracle(scenes.half_disk_scene(g="zero").with_(src_c0=4.0))
    m, v, _ = o.solve(X, 8192, 42)
    check_vs_exact(m, _se(v), 1 - r ** 2, 3e-4, "half disk Poisson")
    k = 3.0
    o = oracle_mod.Oracle(scenes.half_disk_scene(g="zero", sigma=k * k).with_(src_c0=9.0))
    m, v, _ = o.solve(X, 8192, 43)
    check_vs_exact(m, _se(v), 1 - special.i0(k * r) / special.i0(k), 3e-4, "half disk screened source")


def _annulus_exact(r, a, b, k):
    N = lambda s: special.i0(k * s) * special.k1(k * b) + special.k0(k * s) * special.i1(k * b)
    u = N(r) / N(a)
    dN = k * (special.i1(k * a) * special.k1(k * b) - special.k1(k * a) * special.i1(k * b))
    return u, -u * dN / N(a)


def _annulus_points(n, seed, a, b):
    rng = np.random.default_rng(seed)
    r = rng.uniform(a + 0.05, b - 0.05, n)
    t = rng.uniform(0, 2 * np.pi, n)
    return np.stack([r * np.cos(t), r * np.sin(t)], 1), r


def test_annulus_reflecting_outer_wall(oracle_mod):
    """u = 1 on r = a, du/dr = 0 on r = b:
    u = [I0(kr) K1(kb) + K0(kr) I1(kb)] / [same at r = a]."""
    a, b, k = 0.4, 1.0, 2.0
    sc = scenes.annulus_reflecting_scene(a, b, sigma=k * k)
    X, r = _annulus_points(24, 33, a, b)
    m, v, _ = oracle_mod.Oracle(sc).solve(X, 8192, 34)
    u, _ = _annulus_exact(r, a, b, k)
    check_vs_exact(m, _se(v), u, 4e-4, "annulus reflecting")


def test_annulus_reflecting_inner_radius_derivative(oracle_mod):
    """Differential walk on stars (Sec. 4.4): du/da = -u N'(a)/N(a), the nested
    walks reflecting off the outer wall.  Bias budget as for the disk pin:
    the backward-difference offset (delta/2) u_rr and the shell."""
    a, b, k = 0.4, 1.0, 2.0
    sc = scenes.annulus_reflecting_scene(a, b, sigma=k * k, eps=1e-3, delta=1e-2)
    X, r = _annulus_points(24, 35, a, b)
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 4096, 36)
    _, du = _annulus_exact(r, a, b, k)
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), du, 0.05 * np.abs(du).max(), "annulus du/da")


def test_nested_walks_reflect(oracle_mod):
    """The nested walks of a differential terminal are walks on stars too
    (the nesting goes through the Dirichlet boundary only): from a point in
    the shell at the middle of an inner edge the offset point is at radius
    a cos(pi/n) + delta, and the mean of the nested estimates there is the
    annulus solution (without the wall it would be the exterior solution,
    ~0.03 lower at delta = 0.05)."""
    a, b, k, n = 0.4, 1.0, 2.0, 256
    sc = scenes.annulus_reflecting_scene(a, b, n_in=n, sigma=k * k, eps=1e-3, delta=0.05)
    h = math.pi / n
    rmid = a * math.cos(h)
    x = np.array([[(rmid + 4e-4) * math.cos(h), (rmid + 4e-4) * math.sin(h)]])
    rec = oracle_mod.Oracle(sc).walk_records(x, 16384, 45, mode=1, want_udot=False)
    assert np.all(rec["steps"] >= 2)
    uoff = rec["uoff"][0]
    u, _ = _annulus_exact(np.array([rmid + 0.05]), a, b, k)
    check_vs_exact([uoff.mean()], [uoff.std() / math.sqrt(uoff.size)], u, 3e-4, "nested reflect")


def test_half_disk_radius_derivative(oracle_mod):
    """Half disk of radius R with g = 1: the mirror of the disk pin,
    du/dR = -k I0(kr) I1(kR) / I0(kR)^2 (the diameter moves tangentially)."""
    k = 3.0
    sc = scenes.half_disk_scene(sigma=k * k, g="one", eps=1e-3, delta=1e-2)
    X = scenes.points_in_half_disk(24, 37, rmax=0.8)
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 4096, 38)
    r = np.hypot(X[:, 0], X[:, 1])
    exact = -k * special.i0(k * r) * special.i1(k) / special.i0(k) ** 2
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), exact, 0.05 * np.abs(exact).max(), "half disk du/dR")


# ------------------------------------------------- reduction to WoS --------

def test_out_of_reach_wall_reduces_to_walk_on_spheres(oracle_mod):
    """A reflecting segment outside the domain is never within a star radius
    (its silhouette ends lie beyond the Dirichlet distance) and no ray
    reaches it, so without a source each walk-on-stars step draws the same
    direction and roulette numbers as Algorithm 1: the walks coincide."""
    base = scenes.c1_polygon(64, eps=1e-3, delta=1e-2, sigma=4.0, g="one")
    wall = base.with_(NV=np.array([[3.0, -1.0], [3.0, 1.0]]), nsegs=np.array([[0, 1]], np.int32))
    X = scenes.points_in_disk(6, 0.8, 39)
    a = oracle_mod.Oracle(base).walk_records(X, 64, 40, mode=1)
    b = oracle_mod.Oracle(wall).walk_records(X, 64, 40, mode=1)
    for key in ("u", "steps", "prim", "uoff"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(a["udot"], b["udot"])
