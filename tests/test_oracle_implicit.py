"""Pins of the oracle on implicit boundaries (Sec. 7.4): the zero set of
h(x) = c + sum_n a_n / |x - p_n| with the domain {h > 0}.

* The safe radius is safe (h >= 0 on a dense sampling of the disk, for many
  points of a multi-monopole domain) and, for one monopole, equals the
  distance to the circle |x - p| = a / |c|.
* One monopole: the domain is that disk, so the disk's closed forms apply:
  Poisson f = 4, g = 0: u = r0^2 - r^2; harmonic data x^2 - y^2 exactly;
  screened g = 1: I0(k r) / I0(k r0) -- including points next to the pole
  (which the walks must not take for boundary points).
* Parameter derivatives through the level-set normal velocity
  V_n = (dh/dpi) / |grad h|: du/da = 2 a / c^2 and du/dp = 2 (x - p) for
  the Poisson case, the screened du/da, and central differences with common
  random numbers on two overlapping monopoles.
"""
import math

import numpy as np
import pytest
from scipy import special

import scenes
from helpers import check_vs_exact


def _se(v):
    return np.sqrt(np.maximum(np.asarray(v, float), 0))


def _disk_points(n, seed, p, rmax):
    rng = np.random.default_rng(seed)
    r = rmax * np.sqrt(rng.random(n))
    t = 2 * np.pi * rng.random(n)
    return np.stack([p[0] + r * np.cos(t), p[1] + r * np.sin(t)], 1), r


def _h(mono, c, x):
    return c + sum(m[0] / np.hypot(x[..., 0] - m[1], x[..., 1] - m[2]) for m in mono)


def test_safe_radius_is_safe_and_exact_for_one_monopole(oracle_mod):
    mono = np.array([[0.05, -0.3, 0.0], [0.04, 0.25, 0.1], [0.03, 0.0, -0.3], [0.05, 0.05, 0.05]])
    c = -0.4
    sc = scenes.monopole_scene(mono, c=c, src_c0=1.0)
    o = oracle_mod.Oracle(sc)
    rng = np.random.default_rng(4)
    pts = rng.uniform(-0.7, 0.7, (4000, 2))
    pts = pts[_h(mono, c, pts) > 1e-3][:200]
    assert len(pts) == 200
    for x in pts:
        d = o.safe_radius(x)
        assert d > 0
        rr = d * np.sqrt(rng.random(2000))[:, None]
        th = 2 * np.pi * rng.random(2000)[:, None]
        y = x + rr * np.hstack([np.cos(th), np.sin(th)])
        ring = x + d * np.stack([np.cos(np.linspace(0, 2 * np.pi, 720)), np.sin(np.linspace(0, 2 * np.pi, 720))], 1)
        assert _h(mono, c, y).min() > -1e-12 and _h(mono, c, ring).min() > -1e-9
    one = scenes.monopole_scene([[0.5, 0.1, -0.2]], c=-1.0)
    o1 = oracle_mod.Oracle(one)
    X, r = _disk_points(50, 5, (0.1, -0.2), 0.49)
    for x, ri in zip(X, r):
        assert abs(o1.safe_radius(x) - (0.5 - ri)) < 1e-12


def test_one_monopole_poisson_harmonic_screened(oracle_mod):
    p, a, c = (0.1, -0.2), 0.5, -1.0
    r0 = a / -c
    X, r = _disk_points(24, 6, p, 0.45)
    o = oracle_mod.Oracle(scenes.monopole_scene([[a, *p]], c=c, src_c0=4.0))
    m, v, _ = o.solve(X, 8192, 7)
    check_vs_exact(m, _se(v), r0 ** 2 - r ** 2, 3e-4, "monopole Poisson")
    o = oracle_mod.Oracle(scenes.monopole_scene([[a, *p]], c=c, g=(0.0, None, [[1.0, 0.0], [0.0, -1.0]])))
    m, v, _ = o.solve(X, 8192, 8)
    check_vs_exact(m, _se(v), X[:, 0] ** 2 - X[:, 1] ** 2, 3e-4, "monopole harmonic")
    k = 3.0
    o = oracle_mod.Oracle(scenes.monopole_scene([[a, *p]], c=c, sigma=k * k, g=(1.0, None, None)))
    Xn = np.concatenate([X, np.array(p)[None, :] + [[1e-5, 0.0], [0.0, -2e-3]]])
    rn = np.concatenate([r, [1e-5, 2e-3]])
    m, v, _ = o.solve(Xn, 8192, 9)
    check_vs_exact(m, _se(v), special.i0(k * rn) / special.i0(k * r0), 3e-4, "monopole screened")


def test_one_monopole_derivatives(oracle_mod):
    p, a, c = (0.1, -0.2), 0.5, -1.0
    X, r = _disk_points(24, 10, p, 0.4)
    sc = scenes.monopole_scene([[a, *p]], c=c, src_c0=4.0, eps=1e-3, delta=1e-2)
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 4096, 11)
    # u = (a/|c|)^2 - |x - p|^2
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), np.full(len(X), 2 * a / c ** 2), 0.03, "du/da")
    check_vs_exact(jm[:, 1], _se(jv[:, 1]), 2 * (X[:, 0] - p[0]), 0.03, "du/dpx")
    check_vs_exact(jm[:, 2], _se(jv[:, 2]), 2 * (X[:, 1] - p[1]), 0.03, "du/dpy")
    k = 3.0
    sc = scenes.monopole_scene([[a, *p]], c=c, sigma=k * k, g=(1.0, None, None), eps=1e-3, delta=1e-2)
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 4096, 12)
    r0 = a / -c
    exact = -special.i0(k * r) * k * special.i1(k * r0) / special.i0(k * r0) ** 2 / -c
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), exact, 0.05 * np.abs(exact).max(), "screened du/da")


def test_two_monopoles_central_differences(oracle_mod):
    """Central differences in a_1 and p_2x with common random numbers against
    the differential walks' estimate (no closed form for the merged blob)."""
    mono = np.array([[0.3, -0.25, 0.0], [0.25, 0.25, 0.05]])
    c = -1.0
    base = scenes.monopole_scene(mono, c=c, src_c0=4.0, eps=1e-3, delta=1e-2)
    X = np.array([[-0.2, 0.05], [0.0, 0.0], [0.2, -0.05], [0.3, 0.15]])
    W, hh = 16384, 2e-3
    jm, jv, _, _ = oracle_mod.Oracle(base).jvp(X, W, 20)
    for j in (0, 4):
        mp, mm = mono.copy(), mono.copy()
        mp.ravel()[j] += hh
        mm.ravel()[j] -= hh
        up, vp, _ = oracle_mod.Oracle(base.with_(mono=mp)).solve(X, W, 21)
        um, vm, _ = oracle_mod.Oracle(base.with_(mono=mm)).solve(X, W, 21)
        fd = (up - um) / (2 * hh)
        se = np.sqrt(jv[:, j] + (vp + vm) / (2 * hh) ** 2 * 0.05)
        assert np.all(np.abs(jm[:, j] - fd) < 4 * se + 0.05 * np.abs(fd) + 0.01), (j, jm[:, j], fd, se)


def test_harnack_radius(oracle_mod):
    """Harnack's inequality for positive harmonic functions on a 3D ball,
    f(y) >= f(x) R (R - r) / (R + r)^2, on random sums of positive monopoles
    with poles outside the ball; the Harnack radius r of a point makes that
    bound equal -c for f = h - c (R = distance to the nearest pole), so h
    stays positive on the 3D ball of radius r around x (sampled)."""
    rng = np.random.default_rng(13)
    for _ in range(20):
        P = rng.normal(size=(4, 3)) * 2.0
        a = rng.uniform(0.1, 1.0, 4)
        R = np.min(np.linalg.norm(P, axis=1)) * 0.9
        f0 = np.sum(a / np.linalg.norm(P, axis=1))
        y = rng.normal(size=(500, 3))
        y /= np.linalg.norm(y, axis=1)[:, None]
        rr = R * rng.uniform(0, 1, (500, 1))
        fy = np.sum(a / np.linalg.norm((rr * y)[:, None, :] - P[None], axis=2), axis=1)
        bound = f0 * R * (R - rr[:, 0]) / (R + rr[:, 0]) ** 2
        assert np.all(fy >= bound * (1 - 1e-12))
    mono = np.array([[0.05, -0.3, 0.0], [0.04, 0.25, 0.1], [0.03, 0.0, -0.3], [0.05, 0.05, 0.05]])
    c = -0.4
    o = oracle_mod.Oracle(scenes.monopole_scene(mono, c=c))
    pts = rng.uniform(-0.7, 0.7, (4000, 2))
    pts = pts[_h(mono, c, pts) > 1e-3][:100]
    for x in pts:
        r = o.safe_radius(x, harnack=True)
        Rp = np.min(np.hypot(x[0] - mono[:, 1], x[1] - mono[:, 2]))
        f = _h(mono, c, x) - c
        assert abs(f * Rp * (Rp - r) / (Rp + r) ** 2 - (-c)) < 1e-9 * f
        y = rng.normal(size=(400, 3))
        y /= np.linalg.norm(y, axis=1)[:, None]
        q = np.array([x[0], x[1], 0.0]) + r * rng.uniform(0, 1, (400, 1)) ** (1 / 3) * y
        h3 = c + np.sum(mono[:, 0] / np.linalg.norm(q[:, None, :] - np.c_[mono[:, 1:], np.zeros(4)][None], axis=2), 1)
        assert h3.min() > -1e-12


def test_wide_shell_projection(oracle_mod):
    """With a wide shell (eps = 0.03) the boundary value is taken at the
    Newton projection of the stopping point onto the zero set: data
    g = |x - p|^2 equal r0^2 on the circle give u = r0^2 everywhere; the
    projection's error is second order (~1e-4), the stopping point's would be
    first order and one-signed (~2 r0 eta ~ 0.01)."""
    p, a, c = (0.1, -0.2), 0.5, -1.0
    X, r = _disk_points(24, 14, p, 0.4)
    g = (p[0] ** 2 + p[1] ** 2, [-2 * p[0], -2 * p[1]], [[1.0, 0.0], [0.0, 1.0]])
    for sd, (nm, fn) in enumerate([("solve", None), ("joint u of differential walks", "jvp")]):
        sc = scenes.monopole_scene([[a, *p]], c=c, g=g, eps=0.03, delta=0.06)
        o = oracle_mod.Oracle(sc)
        if fn is None:
            m, v, _ = o.solve(X, 8192, 15)
            check_vs_exact(m, _se(v), np.full(len(X), 0.25), 1e-3, "wide shell " + nm)
        else:
            rec = o.walk_records(X, 4096, 16, mode=1, want_udot=False)
            u = rec["u"]
            check_vs_exact(u.mean(1), u.std(1) / np.sqrt(u.shape[1]), np.full(len(X), 0.25), 1e-3,
                           "wide shell " + nm)


def test_restricted_harmonic_data_has_zero_derivative(oracle_mod):
    """Harmonic restricted data x^2 - y^2: u = x^2 - y^2 whatever the shape,
    so every derivative vanishes; the estimator's dg/dn - du/dn cancels up to
    the offset bias (a missing dg/dn leaves -V_n du/dn ~ O(1))."""
    p, a, c = (0.1, -0.2), 0.5, -1.0
    X, r = _disk_points(24, 16, p, 0.4)
    sc = scenes.monopole_scene([[a, *p]], c=c, g=(0.0, None, [[1.0, 0.0], [0.0, -1.0]]), eps=1e-3, delta=1e-2)
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 4096, 17)
    for j in range(3):
        check_vs_exact(jm[:, j], _se(jv[:, j]), np.zeros(len(X)), 0.02, f"harmonic data d/dpi_{j}")


def _grid(lo, hi, n):
    g1 = lo + (np.arange(n) + 0.5) * (hi - lo) / n
    X = np.stack(np.meshgrid(g1, g1), -1).reshape(-1, 2)
    return X, ((hi - lo) / n) ** 2


def test_band_term_is_the_area_derivative_of_a_disk(oracle_mod):
    """Reynolds transport with integrand 1: d(area)/dpi is the boundary
    integral of V_n.  One monopole: the domain is the disk of radius
    r0 = a/|c|, so d(area)/da = 2 pi r0 / |c| and d(area)/dp = 0; the band
    sum (1/eps) sum_band V_n dA approaches it as eps -> 0 (the first-order
    band h/|grad h| < eps is r (r0 - r)/r0 < eps, width ~eps)."""
    a, c, p = 0.5, -1.0, (0.05, -0.1)
    r0 = a / -c
    X, dA = _grid(-0.6, 0.6, 1200)
    o = oracle_mod.Oracle(scenes.monopole_scene([[a, *p]], c=c))
    for eps in (0.02, 0.005):
        g, m = o.band_grad(X, np.full(len(X), dA / eps), eps)
        exact = 2 * np.pi * r0 / -c
        assert abs(g[0] - exact) < (1.5 * eps / r0 + 0.003) * exact, (eps, g[0], exact)
        assert np.all(np.abs(g[1:]) < 0.003 * exact), g
        # the band is the annulus r (r0 - r)/r0 < eps inside the disk
        r = np.hypot(X[:, 0] - p[0], X[:, 1] - p[1])
        inner = r0 / 2 + np.sqrt(r0 ** 2 / 4 - eps * r0)
        away = (np.abs(r - inner) > 1e-3) & (np.abs(r - r0) > 1e-3)
        assert np.array_equal(m[away], np.where((r > inner) & (r < r0), 1, np.where(r < r0, 2, 0))[away])


def test_band_term_matches_finite_differences_of_a_weighted_area(oracle_mod):
    """Two overlapping monopoles, J = integral over the domain of
    f(x) = 1 + x + y^2: dJ/dpi (boundary integral of V_n f) against central
    differences of J counted on the same grid."""
    mono = np.array([[0.3, -0.25, 0.0], [0.25, 0.25, 0.05]])
    c = -1.0
    X, dA = _grid(-0.9, 0.9, 1800)
    f = 1 + X[:, 0] + X[:, 1] ** 2
    eps = 0.004
    g, _ = oracle_mod.Oracle(scenes.monopole_scene(mono, c=c)).band_grad(X, f * dA / eps, eps)
    hh = 4e-3
    for j in range(6):
        mp, mm = mono.copy(), mono.copy()
        mp.ravel()[j] += hh
        mm.ravel()[j] -= hh
        Jp = np.sum(f * (_h(mp, c, X) > 0)) * dA
        Jm = np.sum(f * (_h(mm, c, X) > 0)) * dA
        fd = (Jp - Jm) / (2 * hh)
        assert abs(g[j] - fd) < 0.03 * np.abs(g).max(), (j, g[j], fd)
