"""Pins of the oracle's walk on stars in 3D: reflecting triangle meshes
(Sec. 3.4 eq. (mixed_bvp); differential version Sec. 4.4 eq.
(mixed_bvp_deriv)).

Checked against things fixed outside the oracle:

* silhouette distances worked out by hand on the L-shaped prism (rims and
  the re-entrant edge), and on a reflecting cube from outside by an
  independent rule (an edge is on the contour when one of its faces turns
  towards x and the other away, by the sign of the outward normal);
  star-shapedness against brute-force visibility; ray hits against the two
  walls' planes;
* whole walks against closed forms: the re-entrant edge r^(2/3) cos(2 theta/3)
  (Laplace) and I_{2/3}(k r) cos(2 theta/3) (screened), a quadratic harmonic
  field with zero flux on both walls, the Robin condition with nonzero flux
  on a wall of a cube, mirror symmetry on the half ball and the half ball's
  derivative in its radius, and walks that start on a wall;
* the exact reduction to Algorithm 1 when the reflecting surface is out of
  reach.
"""
import math

import numpy as np
import pytest
from scipy import special

import scenes
from helpers import check_vs_exact


def _se(v):
    return np.sqrt(np.maximum(np.asarray(v, float), 0))


def _cyl(X):
    r = np.hypot(X[:, 0], X[:, 1])
    th = np.mod(np.arctan2(X[:, 1], X[:, 0]), 2 * np.pi)
    return r, th


def _segd(x, a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    t = np.clip(np.dot(x - a, b - a) / np.dot(b - a, b - a), 0, 1)
    return float(np.linalg.norm(x - (a + t * (b - a))))


@pytest.fixture(scope="module")
def lprism(oracle_mod):
    sc = scenes.lprism_scene(n=6, n_wall=6)
    return sc, oracle_mod.Oracle(sc)


# ------------------------------------------------- silhouettes and rays ----

RIMS = [([1, 0, -1], [1, 0, 1]), ([0, -1, -1], [0, -1, 1]), ([0, 0, -1], [1, 0, -1]),
        ([0, 0, 1], [1, 0, 1]), ([0, -1, -1], [0, 0, -1]), ([0, -1, 1], [0, 0, 1])]


def _lprism_silhouette(x):
    """By hand: the walls' rims (edges with one triangle) always count; the
    re-entrant edge (the z axis) counts unless x is in the quadrant x < 0,
    y > 0, from where both walls face x; the edges inside each flat wall
    never do (their two triangles lie on either side of the plane through x
    and the edge)."""
    c = [_segd(x, a, b) for a, b in RIMS]
    if not (x[0] < 0 and x[1] > 0):
        c.append(_segd(x, [0, 0, -1], [0, 0, 1]))
    return min(c)


def test_silhouette_distance_lprism(lprism):
    sc, o = lprism
    for x in scenes.points_in_lprism(300, 5, zlim=0.95):
        assert abs(o.silhouette(x) - _lprism_silhouette(x)) < 1e-12, x


def _wall_triangle(sc, x):
    """Reflecting triangle containing x (brute force)."""
    for i, t in enumerate(sc.nsegs):
        a, b, c = sc.NV[t]
        n = np.cross(b - a, c - a)
        if abs(np.dot(n, x - a)) > 1e-12 * np.linalg.norm(n):
            continue
        M = np.stack([b - a, c - a], 1)
        uv = np.linalg.lstsq(M, x - a, rcond=None)[0]
        if uv.min() >= -1e-12 and uv.sum() <= 1 + 1e-12:
            return i
    raise AssertionError(x)


def test_silhouette_on_the_wall_3d(lprism):
    """x on a wall (domain side given): the re-entrant edge is a silhouette
    (the other wall leaves to the outside of this wall's plane), the wall's
    own inner edges are not (x is in the plane of both their triangles), so
    the distance is to the edge or to a rim, whichever is nearer; also with x
    rounded a hair off the wall's plane."""
    sc, o = lprism
    for s in (0.05, 0.3, 0.7):
        for z in (-0.6, 0.2):
            x = np.array([s, 0.0, z])
            want = min(s, 1 - s, 1 - abs(z))
            assert abs(o.silhouette(x, on=_wall_triangle(sc, x), nin=[0, 1, 0]) - want) < 1e-12
            x = np.array([0.0, -s, z])
            assert abs(o.silhouette(x, on=_wall_triangle(sc, x), nin=[-1, 0, 0]) - want) < 1e-12
    for off in (1e-9, -1e-9):
        x = np.array([0.03, 0.0, 0.1])
        d = o.silhouette(x + [0, off, 0], on=_wall_triangle(sc, x), nin=[0, 1, 0])
        assert abs(d - math.hypot(0.03, off)) < 1e-12


def test_silhouette_of_a_cube_seen_from_outside(oracle_mod):
    """A closed reflecting cube (outward winding) seen from outside: an edge
    is on the contour when exactly one of its two faces has its outward
    normal towards x -- an orientation rule, independent of the oracle's
    plane-side rule; the distance is that to the nearest contour edge.  From
    inside no edge is a silhouette."""
    Vc, Tc = scenes.box_triangles(0.5)
    sc = scenes.sphere_scene(4, R=3.0).with_(NV=Vc, nsegs=Tc)
    o = oracle_mod.Oracle(sc)
    a, b, c = Vc[Tc[:, 0]], Vc[Tc[:, 1]], Vc[Tc[:, 2]]
    nrm = np.cross(b - a, c - a)
    edges = {}
    for i, t in enumerate(Tc):
        for k in range(3):
            e = tuple(sorted((t[k], t[(k + 1) % 3])))
            edges.setdefault(e, []).append(i)
    rng = np.random.default_rng(3)
    for _ in range(200):
        x = rng.uniform(-2, 2, 3)
        if np.abs(x).max() < 0.6:
            continue
        want = np.inf
        for (p, q), f in edges.items():
            front = [np.dot(nrm[j], x - Vc[p]) > 0 for j in f]
            if front[0] != front[1]:
                want = min(want, _segd(x, Vc[p], Vc[q]))
        assert abs(o.silhouette(x, cap=10.0) - want) < 1e-12, x
    for x in rng.uniform(-0.45, 0.45, (50, 3)):
        assert o.silhouette(x, cap=10.0) == 10.0


def _visible(x, y):
    """Does the segment x-y stay in the L-shaped prism (no wall crossing)?"""
    t = np.linspace(0, 1, 400)[1:]
    P = x[None, :] + t[:, None] * (y - x)[None, :]
    return not np.any((P[:, 0] > 0) & (P[:, 1] < 0) & (np.abs(P[:, 2]) <= 1))


def _dirs(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_star_radius_is_star_shaped_3d(lprism):
    """Brute-force visibility: every domain point within the star radius
    min(d_Dirichlet, d_silhouette) is visible from x."""
    sc, o = lprism
    rng = np.random.default_rng(9)
    for x in scenes.points_in_lprism(40, 11, zlim=0.8):
        R = min(o.closest(x)["d"], o.silhouette(x))
        Y = x + R * np.cbrt(rng.random((200, 1))) * _dirs(rng, 200)
        Y = Y[~((Y[:, 0] > 0) & (Y[:, 1] < 0))]
        assert all(_visible(x, y) for y in Y), x


def test_ray_hits_lprism(lprism):
    """Rays against the walls y = 0 (x in [0, 1]) and x = 0 (y in [-1, 0]),
    |z| <= 1, intersected by hand."""
    sc, o = lprism
    rng = np.random.default_rng(12)
    for x in scenes.points_in_lprism(200, 13, zlim=0.9):
        d = _dirs(rng, 1)[0]
        hits = []
        if d[1] != 0:
            t = -x[1] / d[1]
            p = x + t * d
            if t > 0 and 0 <= p[0] <= 1 and abs(p[2]) <= 1:
                hits.append(t)
        if d[0] != 0:
            t = -x[0] / d[0]
            p = x + t * d
            if t > 0 and -1 <= p[1] <= 0 and abs(p[2]) <= 1:
                hits.append(t)
        t, seg = o.ray(x, d, 10.0)
        if hits:
            assert abs(t - min(hits)) < 1e-12 and seg >= 0
        else:
            assert seg == -1 and t == 10.0


# -------------------------------------------------------- closed forms -----

def test_reentrant_edge_laplace_3d(lprism):
    """Lap u = 0 in the L-shaped prism, zero flux on both walls at the
    re-entrant edge, u = r^(2/3) cos(2 theta/3) (independent of z) as mapped
    data on the outer faces and caps.  Bias: the piecewise-linear data on a
    1/6 grid (h^2/8 |g''| < 1e-3 on the faces, larger only in the caps'
    cells at the edge, far from the points) and the shell."""
    sc, o = lprism
    X = scenes.points_in_lprism(12, 21, zlim=0.4)
    m, v, _ = o.solve(X, 2048, 22)
    r, th = _cyl(X)
    check_vs_exact(m, _se(v), scenes.corner_harmonic(r, th), 2e-3, "L-prism Laplace")


def test_reentrant_edge_screened_3d(oracle_mod):
    """Lap u = k^2 u: u = I_{2/3}(k r) cos(2 theta/3); exercises the 3D
    weights of steps that end on a wall."""
    k = 2.0
    g = lambda r, th: special.iv(2.0 / 3.0, k * r) * np.cos(2 * th / 3)
    sc = scenes.lprism_scene(n=6, n_wall=6, sigma=k * k, gfun=g)
    X = scenes.points_in_lprism(12, 23, zlim=0.4)
    m, v, _ = oracle_mod.Oracle(sc).solve(X, 2048, 24)
    r, th = _cyl(X)
    check_vs_exact(m, _se(v), g(r, th), 3e-3, "L-prism screened")


def _lprism_poly(oracle_mod):
    # u = x^2 - y^2 + (2 z^2 - x^2 - y^2)/2: harmonic, du/dy = 0 on y = 0 and
    # du/dx = 0 on x = 0, exact as restricted data
    A = np.diag([0.5, -1.5, 1.0])
    sc = scenes.lprism_scene(n=2, n_wall=4).with_(bc=[scenes._restricted(0.0, None, A, 3)])
    u = lambda X: 0.5 * X[:, 0] ** 2 - 1.5 * X[:, 1] ** 2 + X[:, 2] ** 2
    return sc, oracle_mod.Oracle(sc), u


def test_lprism_quadratic_field(oracle_mod):
    """A quadratic harmonic field with zero flux on both walls, exact as
    restricted data: the only bias is the shell (|grad u| eps ~ 3e-4)."""
    sc, o, u = _lprism_poly(oracle_mod)
    X = scenes.points_in_lprism(16, 25, zlim=0.8)
    m, v, _ = o.solve(X, 4096, 26)
    check_vs_exact(m, _se(v), u(X), 5e-4, "L-prism quadratic")


def test_walks_starting_on_a_wall_3d(oracle_mod):
    """Points on the walls (hemisphere sampling at the start) of the
    quadratic-field problem."""
    sc, o, u = _lprism_poly(oracle_mod)
    X, tri = scenes.points_on_triangles(sc.NV, sc.nsegs, 16, 27)
    m, v, _ = o.solve(X, 4096, 28, start_seg=tri)
    check_vs_exact(m, _se(v), u(X), 5e-4, "L-prism on wall")


def test_robin_wall_of_a_cube(oracle_mod):
    """Cube [-1, 1]^3 with the Robin condition du/dn - mu u = h on the face
    x = -1 (n = +x into the domain): u = 1 + x/2 + x^2 - z^2 has
    du/dn = -3/2 and u = 3/2 - z^2 there, so h = -3/2 - mu (3/2 - z^2);
    Dirichlet data u on the other faces."""
    mu = 0.5
    g = scenes._restricted(1.0, [0.5, 0.0, 0.0], np.diag([1.0, 0.0, -1.0]), 3)
    h = scenes._restricted(-1.5 - mu * 1.5, None, np.diag([0.0, 0.0, mu]), 3)
    # a graded wall grid: triangles of unequal areas (the race weighs them)
    sc = scenes.box_wall_scene(n_wall=3, g=g, robin_mu=mu, robin_h=h, graded=2.0)
    X = np.random.default_rng(29).uniform(-0.85, 0.85, (16, 3))
    m, v, _ = oracle_mod.Oracle(sc).solve(X, 4096, 30)
    u = 1 + 0.5 * X[:, 0] + X[:, 0] ** 2 - X[:, 2] ** 2
    check_vs_exact(m, _se(v), u, 1e-3, "cube Robin")
    # the Neumann data alone (mu = 0): h = du/dn = -3/2
    sc0 = scenes.box_wall_scene(n_wall=3, g=g, robin_h=scenes._restricted(-1.5, dim=3), graded=2.0)
    m, v, _ = oracle_mod.Oracle(sc0).solve(X, 4096, 31)
    check_vs_exact(m, _se(v), u, 1e-3, "cube Neumann data")


def test_robin_boundary_sample_3d_disk_moments(oracle_mod):
    """The Robin boundary sample over the graded wall x = -1 (triangles of
    unequal areas) around a point at height h with radius R: L 1(z in B)
    phi(z) is unbiased for the integral of phi over the disk the ball cuts
    from the wall, of radius a = sqrt(R^2 - h^2): pi a^2 for phi = 1 and
    pi a^2 (h^2 + a^2 / 2) for phi = |z - x|^2.  A race that ignored the
    areas, or points not uniform on their triangle, would miss both."""
    sc = scenes.box_wall_scene(n_wall=3, graded=2.0, robin_mu=1.0)
    o = oracle_mod.Oracle(sc)
    h, R = 0.3, 0.6
    for c in ([-1 + h, 0.1, -0.2], [-1 + h, -0.35, 0.3]):
        x = np.array(c)
        d = o.boundary_sample(x, R, 200000, seed=41)
        inb = d[:, 0] >= 0
        z = d[:, 2:]
        r2 = np.sum((z - x) ** 2, axis=1)
        assert np.all(r2[inb] < R * R)
        a2 = R * R - h * h
        for phi, exact in ((np.ones(len(d)), np.pi * a2), (r2, np.pi * a2 * (h * h + a2 / 2))):
            v = d[:, 1] * inb * phi
            m, se = v.mean(), v.std() / np.sqrt(len(v))
            assert abs(m - exact) < 4 * se, (c, m, exact, se)


def test_half_ball_mirror(oracle_mod):
    """Half ball with a reflecting equatorial disk: data even in y give the
    full ball's solution, x^2 - z^2 (Laplace) and R sinh(kr) / (r sinh kR)
    (screened; inscribed-mesh bias as in the ball pins)."""
    X = scenes.points_in_half_ball(16, 31)
    o = oracle_mod.Oracle(scenes.half_ball_scene(g="x2-z2", eps=1e-4, delta=1e-3))
    m, v, _ = o.solve(X, 4096, 32)
    check_vs_exact(m, _se(v), X[:, 0] ** 2 - X[:, 2] ** 2, 5e-4, "half ball x2-z2")
    k = 2.0
    o = oracle_mod.Oracle(scenes.half_ball_scene(g="one", sigma=k * k))
    m, v, _ = o.solve(X, 4096, 33)
    r = np.linalg.norm(X, axis=1)
    check_vs_exact(m, _se(v), np.sinh(k * r) / (r * np.sinh(k)), 1e-2, "half ball screened")


def test_half_ball_radius_derivative(oracle_mod):
    """Differential walk on stars in 3D: du/dR of the half ball with g = 1
    and sigma = 4, the full ball's (sinh kr / (r sinh kR)) (1 - kR coth kR)
    (the disk moves tangentially); bias budget of the ball pin."""
    k = 2.0
    sc = scenes.half_ball_scene(g="one", sigma=k * k, eps=1e-3, delta=1e-2)
    X = scenes.points_in_half_ball(8, 35, rmax=0.7)
    r = np.linalg.norm(X, axis=1)
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 2048, 36)
    exact = np.sinh(k * r) / (r * np.sinh(k)) * (1 - k / np.tanh(k))
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), exact, 0.06 * np.abs(exact).max(), "half ball du/dR")


def test_out_of_reach_surface_reduces_to_walk_on_spheres(oracle_mod):
    """A reflecting square outside the ball is never within a star radius
    (its rim lies beyond the Dirichlet distance) and no ray reaches it, so
    without a source each walk-on-stars step draws the same direction and
    roulette numbers as Algorithm 1: the walks coincide."""
    base = scenes.sphere_scene(4, g="one", sigma=3.0, eps=1e-3)
    NV, NT = scenes._grid_rect([3.0, -1, -1], [0, 2, 0], [0, 0, 2], 2, 2)
    wall = base.with_(NV=NV, nsegs=NT)
    X = scenes.points_in_ball(6, 0.1, 0.8, 37)
    a = oracle_mod.Oracle(base).walk_records(X, 32, 38, mode=0)
    b = oracle_mod.Oracle(wall).walk_records(X, 32, 38, mode=0)
    assert np.array_equal(a["steps"], b["steps"])
    assert np.allclose(a["u"], b["u"], rtol=0, atol=1e-12)
