"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses an independent
library (rocRAND, scipy), a closed-form solution of the boundary value problem
(Sec. 3.2), a deterministic special case stated by the paper (Sec. 6.3), an
algebraic identity (Sec. 5.3) or finite differences (Sec. 6.1).
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import integrate, special

import scenes
from helpers import check_vs_exact

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- Philox ----

@pytest.fixture(scope="module")
def rocrand_philox():
    hipcc = shutil.which("hipcc")
    if hipcc is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "philox_rr")
    subprocess.check_call([hipcc, "-O1", "--offload-arch=gfx950", "-o", exe,
                           os.path.join(HERE, "pins", "philox_rocrand.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL, cwd=d)
    return exe


def test_philox_matches_rocrand(oracle_mod, rocrand_philox):
    """Philox4x32-10 (Salmon et al. SC'11) against rocRAND's implementation."""
    rng = np.random.default_rng(7)
    rows = rng.integers(0, 2 ** 32, size=(300, 6), dtype=np.uint64).astype(np.uint32)
    rows[0] = 0
    rows[1] = 0xFFFFFFFF
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_philox], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for r, line in zip(rows, out):
        ref = np.array([int(t) for t in line.split()], np.uint32)
        got = oracle_mod.philox(r[:4], r[4:])
        assert np.array_equal(ref, got), (r, ref, got)


# ------------------------------------------------------- Green / Poisson ----

@pytest.mark.parametrize("sigma", [0.0, 0.5, 10.0, 60.0])
@pytest.mark.parametrize("R", [0.01, 0.3, 1.7])
def test_green_integral_identity(oracle_mod, sigma, R):
    """Integral of G over the ball equals (1 - Q(R))/sigma, i.e. the solution of
    -Lap u + sigma u = 1 with zero boundary data at the centre; at sigma = 0 it
    is R^2/(2D).  Pins G's normalisation, its link to Q, and the sign."""
    for D in (2, 3):
        if D == 2:
            f = lambda r: oracle_mod.green(2, sigma, r, R) * 2 * math.pi * r
        else:
            f = lambda r: oracle_mod.green(3, sigma, r, R) * 4 * math.pi * r * r
        val, _ = integrate.quad(f, 0.0, R, limit=200, epsabs=0, epsrel=1e-11)
        Q = oracle_mod.poisson_scale(D, sigma, R)
        expect = R * R / (2 * D) if sigma == 0 else (1 - Q) / sigma
        assert val == pytest.approx(expect, rel=1e-8, abs=1e-14), (D, sigma, R)
        assert oracle_mod.green(D, sigma, R, R) == pytest.approx(0.0, abs=1e-12)


def test_green_poisson_vs_scipy(oracle_mod):
    """Closed forms of G and Q against scipy.special Bessel functions (2D) and
    the r -> 0 singularity of the free-space kernel."""
    for sigma in (0.3, 4.0, 10.0, 25.0):
        k = math.sqrt(sigma)
        for R in (0.05, 0.4, 1.3):
            assert oracle_mod.poisson_scale(2, sigma, R) == pytest.approx(1 / special.i0(k * R), rel=1e-12)
            assert oracle_mod.poisson_scale(3, sigma, R) == pytest.approx(k * R / math.sinh(k * R), rel=1e-12)
            for r in (1e-4 * R, 0.3 * R, 0.9 * R):
                g2 = (special.k0(k * r) - special.k0(k * R) * special.i0(k * r) / special.i0(k * R)) / (2 * math.pi)
                assert oracle_mod.green(2, sigma, r, R) == pytest.approx(g2, rel=1e-10)
    # singular behaviour: 2D ~ -ln(r)/(2 pi), 3D ~ 1/(4 pi r)
    r = 1e-9
    assert oracle_mod.green(2, 4.0, r, 1.0) * 2 * math.pi / (-math.log(r)) == pytest.approx(1.0, rel=0.1)
    assert oracle_mod.green(3, 4.0, r, 1.0) * 4 * math.pi * r == pytest.approx(1.0, rel=1e-6)
    for D in (2, 3):
        assert oracle_mod.poisson_scale(D, 0.0, 0.7) == 1.0


# ---------------------------------------------------------- closest point ---

def test_closest_point_vs_dense_sampling(oracle_mod):
    """Brute-force closest point against a dense sampling of every primitive:
    never farther than any sample, never closer than the sampling resolution
    allows, and consistent barycentrics."""
    rng = np.random.default_rng(3)
    sc = scenes.c2_star(n=64)
    o = oracle_mod.Oracle(sc)
    t = np.linspace(0, 1, 201)
    segs = sc.V[sc.prims]                                        # (np, 2, 2)
    samp = segs[:, :1, :] * (1 - t)[None, :, None] + segs[:, 1:, :] * t[None, :, None]
    samp = samp.reshape(-1, 2)
    for x in rng.uniform(-1.3, 1.3, (50, 2)):
        h = o.closest(x)
        ds = np.sqrt(((samp - x) ** 2).sum(1)).min()
        assert h["d"] <= ds + 1e-12
        assert h["d"] >= ds - 0.06 / 200
        q = h["bary"][0] * sc.V[sc.prims[h["prim"], 0]] + h["bary"][1] * sc.V[sc.prims[h["prim"], 1]]
        assert np.allclose(q, h["xbar"][:2], atol=1e-12)
        assert abs(np.linalg.norm(x - q) - h["d"]) < 1e-12
    V, T = scenes.icosphere(2)
    s3 = scenes.sphere_scene(2)
    o3 = oracle_mod.Oracle(s3)
    u = np.linspace(0, 1, 41)
    A, B = np.meshgrid(u, u)
    m = A + B <= 1
    a, b = A[m], B[m]
    tri = V[T]
    samp3 = (tri[:, 0:1] * (1 - a - b)[None, :, None] + tri[:, 1:2] * a[None, :, None]
             + tri[:, 2:3] * b[None, :, None]).reshape(-1, 3)
    for x in rng.uniform(-1.4, 1.4, (40, 3)):
        h = o3.closest(x)
        ds = np.sqrt(((samp3 - x) ** 2).sum(1)).min()
        assert h["d"] <= ds + 1e-12
        assert h["d"] >= ds - 0.7 / 40
        tv = V[T[h["prim"]]]
        q = (h["bary"][:, None] * tv).sum(0)
        assert np.allclose(q, h["xbar"], atol=1e-12)
        assert np.all(h["bary"] >= -1e-12) and abs(h["bary"].sum() - 1) < 1e-12


# ------------------------------------------------------- closed forms -------

def _se(v):
    return np.sqrt(np.maximum(v, 0))


def test_harmonic_field_exact_on_polygon(oracle_mod):
    """sigma = 0, restricted g = x^2 - y^2 (harmonic): u = x^2 - y^2 exactly on
    any domain, so only the eps-shell bias (|grad u| eps) remains."""
    sc = scenes.c1_polygon(128)
    X = scenes.points_in_disk(64, 0.9, 1)
    m, v, _ = oracle_mod.Oracle(sc).solve(X, 512, 2)
    check_vs_exact(m, _se(v), X[:, 0] ** 2 - X[:, 1] ** 2, 2 * 2 * sc.eps, "P4")


def test_poisson_source_disk_and_ball(oracle_mod):
    """Source path and PDE sign: -Lap u = f, g = 0 gives u = f (R^2 - r^2)/(2D);
    screened: u = (f/sigma)(1 - I0(kr)/I0(kR)) in 2D."""
    o = oracle_mod.Oracle(scenes.c1_polygon(512, g="one", eps=1e-4).with_(
        bc=[dict(kind="restricted", c=0.0, b=np.zeros(2), A=np.zeros((2, 2)))], src_c0=4.0))
    X = scenes.points_in_disk(24, 0.9, 11)
    r = np.linalg.norm(X, axis=1)
    m, v, _ = o.solve(X, 2048, 5)
    check_vs_exact(m, _se(v), 1 - r ** 2, 5e-4, "P3 disk sigma=0")
    sigma = 10.0
    k = math.sqrt(sigma)
    o = oracle_mod.Oracle(scenes.c1_polygon(512, g="one", eps=1e-4, sigma=sigma).with_(
        bc=[dict(kind="restricted", c=0.0, b=np.zeros(2), A=np.zeros((2, 2)))], src_c0=4.0))
    m, v, _ = o.solve(X, 2048, 6)
    check_vs_exact(m, _se(v), (4.0 / sigma) * (1 - special.i0(k * r) / special.i0(k)), 5e-4,
                   "P3 disk sigma=10")
    # ball (icosphere nu=8: inscribed mesh sits up to ~3.5e-3 inside the sphere)
    o = oracle_mod.Oracle(scenes.sphere_scene(8, g="zero", eps=1e-3, source_c0=6.0))
    X3 = scenes.points_in_ball(8, 0.0, 0.8, 12)
    r3 = np.linalg.norm(X3, axis=1)
    m, v, _ = o.solve(X3, 1024, 7)
    check_vs_exact(m, _se(v), 1 - r3 ** 2, 1e-2, "P3 ball")


def test_screened_constant_data_disk_and_ball(oracle_mod):
    """Russian roulette and Q: g = 1, sigma > 0 gives u = I0(kr)/I0(kR) (disk)
    and R sinh(kr)/(r sinh(kR)) (ball)."""
    sigma = 10.0
    k = math.sqrt(sigma)
    o = oracle_mod.Oracle(scenes.c1_polygon(512, g="one", eps=1e-4, sigma=sigma))
    X = scenes.points_in_disk(32, 0.9, 21)
    r = np.linalg.norm(X, axis=1)
    m, v, _ = o.solve(X, 4096, 8)
    check_vs_exact(m, _se(v), special.i0(k * r) / special.i0(k), 5e-4, "P5 disk")
    sigma = 4.0
    k = 2.0
    o = oracle_mod.Oracle(scenes.sphere_scene(8, g="one", eps=1e-3, sigma=sigma))
    X3 = scenes.points_in_ball(8, 0.1, 0.8, 22)
    r3 = np.linalg.norm(X3, axis=1)
    m, v, _ = o.solve(X3, 1024, 9)
    check_vs_exact(m, _se(v), np.sinh(k * r3) / (r3 * np.sinh(k)), 1e-2, "P5 ball")


def test_shape_derivative_disk(oracle_mod):
    """Differential WoS (Alg. 2) on the disk with g = 1, parameter = radius:
    du/dR = -k I0(kr) I1(kR) / I0(kR)^2.  Bias budget: backward-difference
    offset (delta/2) u_rr ~ 0.04 relative, polygon and shell terms."""
    sigma = 10.0
    k = math.sqrt(sigma)
    sc = scenes.c1_polygon(512, g="one", eps=1e-3, delta=1e-2, sigma=sigma)
    X = scenes.points_in_disk(32, 0.8, 31)
    r = np.linalg.norm(X, axis=1)
    jm, jv, um, _ = oracle_mod.Oracle(sc).jvp(X, 4096, 10)
    exact = -k * special.i0(k * r) * special.i1(k) / special.i0(k) ** 2
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), exact, 0.045 * np.abs(exact).max(), "P6 disk")


def test_shape_derivative_ball(oracle_mod):
    """du/dR for the ball with g = 1: (sinh kr/(r sinh kR)) (1 - kR coth kR)."""
    sigma, k = 4.0, 2.0
    sc = scenes.sphere_scene(8, g="one", eps=1e-3, delta=1e-2, sigma=sigma)
    X3 = scenes.points_in_ball(6, 0.1, 0.7, 32)
    r = np.linalg.norm(X3, axis=1)
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X3, 1024, 11)
    exact = np.sinh(k * r) / (r * np.sinh(k)) * (1 - k / np.tanh(k))
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), exact, 0.06 * np.abs(exact).max(), "P6 ball")


def test_restricted_harmonic_field_has_zero_shape_derivative(oracle_mod):
    """Restricted harmonic data: u = g everywhere, so du/dR = 0; the estimator's
    dg/dn - du/dn cancels up to the offset bias (delta/2) d2g/dn2 V_n.  A
    missing or halved dg/dn term leaves -dg/dn V_n ~ O(1) instead."""
    sc = scenes.c1_polygon(128, eps=1e-3, delta=1e-2)
    X = scenes.points_in_disk(32, 0.9, 41)
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 4096, 12)
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), np.zeros(len(X)), 0.015, "P6 restricted")


def _rotation_params(sc):
    """Replace the parameter by a rigid rotation angle: dv_i/dphi = (-y_i, x_i)."""
    V = sc.V
    return sc.with_(N=1, rowptr=np.arange(sc.nv + 1, dtype=np.int64),
                    pid=np.zeros(sc.nv, np.int32), vel=np.stack([-V[:, 1], V[:, 0]], 1))


def test_rotation_derivative_mapped_and_restricted(oracle_mod):
    """Rotating the boundary by phi: with mapped data the values ride along, so
    u(x; phi) = U(R(-phi) x) and du/dphi = grad u . (y, -x) = 4xy for
    u ~ x^2 - y^2; the velocity is tangential, which exercises the surface
    gradient term of the mapped boundary derivative.  With restricted data
    the field stays put and the (circular) domain does not change: du/dphi = 0."""
    X = scenes.points_in_disk(32, 0.8, 43)
    sc = _rotation_params(scenes.c1_polygon(128, mapped=True, eps=1e-3, delta=1e-2))
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 2048, 14)
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), 4 * X[:, 0] * X[:, 1], 4e-3, "rotation mapped")
    sc = _rotation_params(scenes.c1_polygon(128, eps=1e-3, delta=1e-2))
    jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 2048, 15)
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), np.zeros(len(X)), 0.015, "rotation restricted")


def test_derivative_splits_by_barycentrics(oracle_mod):
    """Explicit surface (Sec. 3.1.2): the velocity at a terminal point is the
    barycentric blend of its primitive's vertex velocities, so with one radial
    parameter per vertex the two vertices of the terminal edge receive udot in
    the ratio b0 (n.u0) : b1 (n.u1), with b the position of the terminal point
    along the edge (computed here from the geometry)."""
    sc = scenes.c1_polygon(12, g="one", eps=1e-3, delta=1e-2, sigma=2.0)
    n = sc.nv
    U = sc.V / np.linalg.norm(sc.V, axis=1, keepdims=True)
    sc = sc.with_(N=n, rowptr=np.arange(n + 1, dtype=np.int64), pid=np.arange(n, dtype=np.int32), vel=U)
    X = scenes.points_in_disk(8, 0.7, 44)
    rec = oracle_mod.Oracle(sc).walk_records(X, 64, 16, mode=1)
    checked = 0
    for p in range(len(X)):
        for m in range(64):
            pr = rec["prim"][p, m]
            if pr < 0:
                continue
            i0, i1 = sc.prims[pr]
            a, b = sc.V[i0], sc.V[i1]
            xb = rec["xbar"][p, m, :2]
            b1 = np.dot(xb - a, b - a) / np.dot(b - a, b - a)
            t = (b - a) / np.linalg.norm(b - a)
            nrm = np.array([t[1], -t[0]])
            ud = rec["udot"][p, m]
            others = np.delete(ud, [i0, i1])
            assert np.all(others == 0.0)
            w0, w1 = (1 - b1) * np.dot(nrm, U[i0]), b1 * np.dot(nrm, U[i1])
            # ud[i0] * w1 == ud[i1] * w0, in a form that is safe near the vertices
            assert abs(ud[i0] * w1 - ud[i1] * w0) <= 1e-9 * (abs(ud[i0]) + abs(ud[i1]) + 1e-300)
            checked += 1
    assert checked > 100


def test_mapped_data_shape_derivative(oracle_mod):
    """Mapped vertex values g_i = x_i^2 - y_i^2 under radial scaling: the
    solution scales as u(x; R) = U(x/R), so du/dR = -x.grad u / R, which for
    u ~ x^2 - y^2 is -2 (x^2 - y^2) / R (Appendix A with V_t kept)."""
    sc = scenes.c1_polygon(128, mapped=True, eps=1e-4, delta=1e-3)
    X = scenes.points_in_disk(32, 0.8, 42)
    jm, jv, um, _ = oracle_mod.Oracle(sc).jvp(X, 2048, 13)
    exact = -2 * (X[:, 0] ** 2 - X[:, 1] ** 2)
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), exact, 2e-3 + 1e-3, "mapped dudR")


def test_annulus_laplace_value_and_derivative(oracle_mod):
    """2D annulus, u = 1 on r = a, 0 on r = b: u = ln(r/b)/ln(a/b) and
    du/da = -ln(r/b)/(a ln(a/b)^2) (mixed labels, parameter on one label)."""
    a, b = 0.4, 1.2
    sc = scenes.annulus_scene(a, b, n=512, eps=1e-3, delta=1e-2)
    rng = np.random.default_rng(51)
    rr = rng.uniform(0.55, 1.0, 24)
    th = rng.uniform(0, 2 * np.pi, 24)
    X = np.stack([rr * np.cos(th), rr * np.sin(th)], 1)
    o = oracle_mod.Oracle(sc)
    m, v, _ = o.solve(X, 2048, 14)
    check_vs_exact(m, _se(v), np.log(rr / b) / np.log(a / b), 3e-3, "P7 annulus u")
    jm, jv, _, _ = o.jvp(X, 4096, 15)
    exact = -np.log(rr / b) / (a * np.log(a / b) ** 2)
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), exact, 0.05 * np.abs(exact).max(), "P7 annulus du/da")


def test_shell_screened_value_and_derivative(oracle_mod):
    """3D screened shell (the shape-from-diffusion layout: emitter inside an
    absorbing outer boundary): u = a sinh(k(b-r)) / (r sinh(k(b-a))) and its
    derivative with respect to the inner radius a."""
    a, b, sigma = 0.5, 1.5, 4.0
    k = 2.0
    sc = scenes.shell_scene(6, 6, a, b, sigma, eps=2e-3, delta=2e-2)
    X = scenes.points_in_ball(8, 0.7, 1.2, 52)
    r = np.linalg.norm(X, axis=1)
    o = oracle_mod.Oracle(sc)
    m, v, _ = o.solve(X, 1024, 16)
    check_vs_exact(m, _se(v), a * np.sinh(k * (b - r)) / (r * np.sinh(k * (b - a))), 2.5e-2, "P7 shell u")
    jm, jv, _, _ = o.jvp(X, 1024, 17)
    s = np.sinh(k * (b - a))
    exact = (np.sinh(k * (b - r)) / r) * (1 / s + a * k * np.cosh(k * (b - a)) / s ** 2)
    check_vs_exact(jm[:, 0], _se(jv[:, 0]), exact, 0.12 * np.abs(exact).max(), "P7 shell du/da")


# --------------------------------------------- deterministic special cases --

def test_offset_inside_shell_gives_zero_normal_derivative(oracle_mod):
    """delta < eps: the nested walk stops at its first query and returns
    g(xbar), so the normal-derivative estimate is identically 0 (Sec. 6.3); with
    g = 1 every udot is exactly 0 and each nested walk costs one query."""
    sc = scenes.c1_polygon(128, g="one", eps=1e-3, delta=5e-4, sigma=2.0)
    X = scenes.points_in_disk(16, 0.8, 61)
    o = oracle_mod.Oracle(sc)
    rec = o.walk_records(X, 64, 18, mode=1)
    prim_rec = o.walk_records(X, 64, 18, mode=0)
    assert np.all(rec["udot"] == 0.0)
    term = rec["prim"] >= 0
    assert term.any() and (~term).any()
    # primal steps of the same stream plus exactly one nested query per terminal walk
    assert np.array_equal(rec["steps"], prim_rec["steps"] + term.astype(np.int64))
    assert np.all(rec["uoff"][term] == 1.0)


def test_no_roulette_without_screening(oracle_mod):
    """sigma = 0 gives alpha = 1, so Russian roulette never stops a walk."""
    sc = scenes.c1_polygon(128)
    X = scenes.points_in_disk(16, 0.9, 62)
    rec = oracle_mod.Oracle(sc).walk_records(X, 64, 19, mode=1)
    assert np.all(rec["prim"] >= 0)


def test_joint_estimate_equals_forward_walk(oracle_mod):
    """The differential walk takes the forward walk's steps with the same random
    numbers (Sec. 5.1, observation 2), so its joint u equals the forward u."""
    sc = scenes.c2_star(n=256)
    X = scenes.star_points(16, 63)
    o = oracle_mod.Oracle(sc)
    a = o.walk_records(X, 32, 20, mode=0)
    b = o.walk_records(X, 32, 20, mode=1, want_udot=False)
    assert np.array_equal(a["u"], b["u"])


# ----------------------------------------------------- estimator algebra ----

def test_ustat_matches_unrolled_pair_sum(oracle_mod):
    """Reverse-mode squared loss: the oracle's O(B) form (eq. ustatistics) equals
    the unrolled sum over ordered pairs m != m' (eq. ustatistics_unrolled)."""
    sc = scenes.c2_star(n=128, kmax=4)
    X = scenes.star_points(6, 64)
    uref = np.linspace(-0.2, 0.3, 6)
    W, B = 16, 8
    o = oracle_mod.Oracle(sc)
    L, g, um, _ = o.grad_sqloss(X, uref, W, B, 21)
    rec = o.walk_records(X, W, 21, mode=1)
    u, ud = rec["u"], rec["udot"]
    expect = np.zeros(sc.N)
    for p in range(len(X)):
        acc = np.zeros(sc.N)
        for b in range(W // B):
            idx = range(b * B, (b + 1) * B)
            pair = np.zeros(sc.N)
            for m in idx:
                for mp in idx:
                    if m != mp:
                        pair += u[p, m] * ud[p, mp]
            acc += pair / (B * (B - 1)) - uref[p] * ud[p, list(idx)].mean(0)
        expect += acc / (W // B)
    assert np.allclose(g, expect, rtol=1e-12, atol=1e-12)
    assert L == pytest.approx(0.5 * ((u.mean(1) - uref) ** 2).sum(), rel=1e-12)
    with pytest.raises(ValueError):
        o.grad_sqloss(X, uref, 12, 8, 21)


def test_reverse_mode_is_weighted_forward_mode(oracle_mod):
    """sum_p w_p udot(x_p) from the reverse accumulation equals the weighted
    sum of the per-point forward-mode means of the same walks."""
    sc = scenes.c2_star(n=128, kmax=4)
    X = scenes.star_points(8, 65)
    w = np.random.default_rng(0).normal(size=8)
    o = oracle_mod.Oracle(sc)
    g, _, _ = o.grad(X, w, 32, 22)
    jm, _, _, _ = o.jvp(X, 32, 22)
    assert np.allclose(g, w @ jm, rtol=1e-11, atol=1e-13)


def test_ustat_unbiased_against_independent_estimates(oracle_mod):
    """E[U-stat gradient] = sum_p (u_p - uref_p) udot_p: compare with the
    product of independent large-sample estimates of u and udot."""
    sc = scenes.c2_star(n=128, kmax=2, eps=2e-3, delta=2e-2)
    X = scenes.star_points(4, 66)
    uref = np.zeros(4)
    o = oracle_mod.Oracle(sc)
    reps = [o.grad_sqloss(X, uref, 64, 8, 1000 + s)[1] for s in range(24)]
    reps = np.array(reps)
    gm, gse = reps.mean(0), reps.std(0, ddof=1) / math.sqrt(len(reps))
    um, uv, _ = o.solve(X, 16384, 77)
    jm, jv, _, _ = o.jvp(X, 16384, 78)
    ref = ((um - uref)[:, None] * jm).sum(0)
    refse = np.sqrt((((um - uref)[:, None] ** 2) * jv).sum(0) + (uv[:, None] * jm ** 2).sum(0))
    z = (gm - ref) / np.sqrt(gse ** 2 + refse ** 2)
    assert np.all(np.abs(z) < 4.5), z


def test_central_difference_with_common_random_numbers(oracle_mod):
    """Sec. 6.1: derivatives agree with finite differences.  Central differences
    with common random numbers, h = 1e-3, against forward-mode udot."""
    sc = scenes.c2_star(n=256, kmax=4, eps=2e-4, delta=2e-3, sigma=10.0)
    X = scenes.star_points(8, 67)
    W = 8192
    o = oracle_mod.Oracle(sc)
    jm, jv, _, _ = o.jvp(X, W, 23)
    h = 1e-3
    for j in (0, 3, 5):
        e = np.zeros(sc.N)
        e[j] = h
        up = oracle_mod.Oracle(sc, V=scenes.vertices_at(sc, sc.pi0 + e)).walk_records(X, W, 24)["u"]
        dn = oracle_mod.Oracle(sc, V=scenes.vertices_at(sc, sc.pi0 - e)).walk_records(X, W, 24)["u"]
        fd = (up - dn) / (2 * h)
        fm, fse = fd.mean(1), fd.std(1, ddof=1) / math.sqrt(W)
        z = (fm - jm[:, j]) / np.sqrt(fse ** 2 + jv[:, j])
        assert np.all(np.abs(z) < 4.0), (j, z, fm, jm[:, j])
        assert abs(np.mean(z)) < 4.0 / math.sqrt(len(z)) + 0.5, (j, z)


def test_nested_walks_skipped_where_boundary_is_static(oracle_mod):
    """Shell a < r < b with only the inner sphere moving: walks that end on
    the static outer sphere run no nested walks (their mean enters every
    derivative times V_n = 0), report the boundary value as the nested mean
    and give a zero derivative; walks ending on the inner sphere do run them."""
    sc = scenes.shell_scene(8, 8, 0.5, 1.0, 4.0, eps=1e-3, delta=1e-2)
    X = scenes.points_in_ball(16, 0.6, 0.9, 91)
    r = oracle_mod.Oracle(sc).walk_records(X, 64, 92, mode=1)
    term = r["prim"] >= 0
    outer = term & (sc.label[np.maximum(r["prim"], 0)] == 0)
    inner = term & (sc.label[np.maximum(r["prim"], 0)] == 1)
    assert outer.sum() > 50 and inner.sum() > 50
    assert np.all(r["uoff"][outer] == 0.0)        # g = 0 on the outer sphere
    assert np.all(r["udot"][outer] == 0.0)
    # no nested walks: a main walk alone rarely takes fewer queries than
    # main + nested; compare with the forward walk of the same stream
    rf = oracle_mod.Oracle(sc).walk_records(X, 64, 92, mode=0)
    assert np.array_equal(r["steps"][outer], rf["steps"][outer])
    assert np.all(r["steps"][inner] > rf["steps"][inner])


def test_vertex_value_parameters_sum_to_constant_data_solution(oracle_mod):
    """Mapped data whose only parameters are the vertex values g_i (no vertex
    moves): u is linear in the g_i, so sum_i du/dg_i is the solution for
    g = 1 -- I0(kr)/I0(kR) on the disk (1 at sigma = 0).  Every terminal
    depends on a parameter through its values alone."""
    n = 256
    for sigma in (0.0, 10.0):
        base = scenes.c1_polygon(n, mapped=True, g="one", eps=1e-3, delta=1e-2, sigma=sigma)
        sc = base.with_(N=n, rowptr=np.zeros(n + 1, np.int64), pid=np.zeros(0, np.int32),
                        vel=np.zeros((0, 2)), bc_pid=np.arange(n, dtype=np.int32))
        X = scenes.points_in_disk(16, 0.8, 93)
        jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 2048, 94)
        tot = jm.sum(axis=1)
        # the per-walk sum has its own variance: estimate it from the mean
        # and per-parameter variances conservatively (parameters of one walk
        # are correlated), via an independent second run
        jm2, _, _, _ = oracle_mod.Oracle(sc).jvp(X, 2048, 95)
        se = np.abs(tot - jm2.sum(axis=1)) / np.sqrt(2) + 1e-3
        k = math.sqrt(sigma)
        r = np.linalg.norm(X, axis=1)
        exact = special.i0(k * r) / special.i0(k) if sigma > 0 else np.ones(len(X))
        assert np.all(np.abs(tot - exact) < 4 * se + 0.01), (sigma, tot - exact)
