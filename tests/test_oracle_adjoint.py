"""The oracle's adjoint formulation of the shape derivative (Appendix B,
eq. (functional_deriv_adjoint)), pinned to closed forms.

J = int_Omega 1/2 (u - uref)^2 with a constant uref = c0.  With independent
walks for the adjoint lambda and for u at the offset point y - delta n, the
estimator's expectation at a finite delta is, per boundary point,
  lambda(y - delta n) / delta * udot(y; u(y - delta n)) + 1/2 (g - c0)^2 V_n
with the exact lambda and u, so each case below checks the mean over many
walks against that expression (statistical, 4.5 standard errors plus the
polygon's discretisation), and the per-walk records against lambda and u at
the offset point:

* disk, -Lap u = 4, g = 0: u = R^2 - r^2, lambda = A (R^2 - r^2) + B (R^4 - r^4)
  with A = (R^2 - c0)/4, B = -1/16; the delta -> 0 limit pi R (R^2 - c0)^2 is
  the derivative of J = pi/6 [(R^2 - c0)^3 + c0^3].
* screened disk (sigma = k^2, roulette), g = 1: u = I0(kr)/I0(kR),
  lambda = -r I1(kr) / (2 k I0(kR)) - c0/k^2 + C I0(kr) (zero at R).
* mapped data on the disk, g = x^2 - y^2 carried by the vertices: u = x^2 - y^2,
  lambda = -c0 (R^2 - r^2)/4 + r^2 (R^2 - r^2) cos(2 theta)/12; the boundary
  value is -V_n du/dn.
* ball (icosphere), -Lap u = 6, g = 0: u = R^2 - r^2,
  lambda = A (R^2 - r^2) + B (R^4 - r^4) with A = (R^2 - c0)/6, B = -1/20.
* A dropped l(g) V_n term, a sign error in lambda or a missing 1/delta each
  move these means by many standard errors.
"""
import numpy as np
import pytest
from scipy import special

import scenes

pytestmark = pytest.mark.filterwarnings("ignore")


@pytest.fixture(scope="module")
def oracle():
    import oracle as o
    o.build(force=False)
    return o


def _disk_poisson(n=128, delta=0.2, K=1, f=4.0):
    return scenes.c1_polygon(n, eps=1e-4, delta=delta, K=K).with_(bc=[scenes._restricted(0.0, dim=2)], src_c0=f)


def _ref(c0, D=2):
    return np.concatenate([[c0], np.zeros(D + D * D)])


def _run(oracle, sc, S, W, seed, c0, reps=4):
    code, bary, wq = scenes.boundary_samples(sc, S, seed)
    o = oracle.Oracle(sc)
    gs, lam, uoff = [], [], []
    for r in range(reps):
        g, l, u, _ = o.adjoint_grad(code, bary, wq, _ref(c0, sc.dim), W, 1000 * seed + r)
        gs.append(g[0])
        lam.append(l)
        uoff.append(u)
    gs = np.array(gs)
    return gs.mean(), gs.std(ddof=1) / np.sqrt(reps), np.concatenate(lam).ravel(), np.concatenate(uoff).ravel()


def _close(mean, se, exact, rel=0.0, z=4.5, what=""):
    print(f"{what}: {mean:.6g} +- {se:.2g} vs {exact:.6g} (z = {(mean - exact) / se:.2f})")
    assert abs(mean - exact) <= z * se + rel * abs(exact), (what, mean, se, exact)


def test_disk_poisson(oracle):
    R, c0, delta = 1.0, 0.5, 0.2
    sc = _disk_poisson(delta=delta)
    m, se, lam, uoff = _run(oracle, sc, 1500, 16, 1, c0)
    r = R - delta
    lam_x = (R * R - c0) / 4 * (R * R - r * r) - (R ** 4 - r ** 4) / 16
    u_x = R * R - r * r
    _close(lam.mean(), lam.std() / np.sqrt(lam.size), lam_x, 0.01, what="lambda")
    _close(uoff.mean(), uoff.std() / np.sqrt(uoff.size), u_x, 0.01, what="u")
    exact = 2 * np.pi * R * (lam_x * u_x / delta ** 2 + 0.5 * c0 ** 2)
    _close(m, se, exact, 0.01, what="dJ/dR at delta")


def test_disk_poisson_limit(oracle):
    """Small delta: the derivative itself, pi R (R^2 - c0)^2, within the
    O(delta) bias of the two backward differences."""
    R, c0, delta = 1.0, 0.25, 0.02
    m, se, _, _ = _run(oracle, _disk_poisson(delta=delta, K=4), 3000, 32, 2, c0)
    exact = np.pi * R * (R * R - c0) ** 2
    _close(m, se, exact, 3 * delta, what="dJ/dR limit")


def test_screened_disk(oracle):
    R, c0, delta, k = 1.0, 0.3, 0.2, 3.0
    sc = scenes.c1_polygon(128, g="one", eps=1e-4, delta=delta, sigma=k * k)
    m, se, lam, uoff = _run(oracle, sc, 1500, 16, 3, c0)
    r = R - delta
    C = (R * special.i1(k * R) / (2 * k * special.i0(k * R)) + c0 / k ** 2) / special.i0(k * R)
    lam_x = -r * special.i1(k * r) / (2 * k * special.i0(k * R)) - c0 / k ** 2 + C * special.i0(k * r)
    u_x = special.i0(k * r) / special.i0(k * R)
    _close(lam.mean(), lam.std() / np.sqrt(lam.size), lam_x, 0.01, what="lambda")
    _close(uoff.mean(), uoff.std() / np.sqrt(uoff.size), u_x, 0.01, what="u")
    exact = 2 * np.pi * R * (lam_x / delta * (-(1.0 - u_x) / delta) + 0.5 * (1.0 - c0) ** 2)
    _close(m, se, exact, 0.01, what="dJ/dR at delta")


def test_mapped_disk(oracle):
    c0, delta = 0.4, 0.2
    sc = scenes.c1_polygon(256, mapped=True, eps=1e-4, delta=delta)
    m, se, _, _ = _run(oracle, sc, 2000, 16, 4, c0)
    r = 1.0 - delta
    a2 = r * r * (1 - r * r) / 12
    beta = (1 - r * r) / delta
    exact = -np.pi * a2 * beta / delta + np.pi / 2 + np.pi * c0 ** 2
    _close(m, se, exact, 0.01, what="mapped dJ/dR at delta")


def test_ball(oracle):
    """c0 = -1 keeps the adjoint's source u - c0 positive: with a source
    that changes sign, lambda is a small difference of two terms and the
    icosphere's O(h^2) deviation from the ball (u 2% low at the offset
    radius here) is amplified several times.  The mesh's own area replaces
    4 pi R^2; 6% covers the rest of the discretisation."""
    R, c0, delta = 1.0, -1.0, 0.2
    sc = scenes.sphere_scene(6, g="zero", eps=1e-4, delta=delta, source_c0=6.0)
    m, se, lam, uoff = _run(oracle, sc, 400, 8, 5, c0)
    r = R - delta
    lam_x = (R * R - c0) / 6 * (R * R - r * r) - (R ** 4 - r ** 4) / 20
    u_x = R * R - r * r
    _close(lam.mean(), lam.std() / np.sqrt(lam.size), lam_x, 0.06, what="lambda")
    _close(uoff.mean(), uoff.std() / np.sqrt(uoff.size), u_x, 0.04, what="u")
    area = scenes.boundary_samples(sc, 1, 0)[2].sum()
    exact = area * (lam_x * u_x / delta ** 2 + 0.5 * c0 ** 2)
    _close(m, se, exact, 0.06, what="ball dJ/dR at delta")


def test_errors(oracle):
    sc = _disk_poisson()
    o = oracle.Oracle(sc)
    code, bary, wq = scenes.boundary_samples(sc, 4, 1)
    with pytest.raises(ValueError):
        o.adjoint_grad(code + 2 * sc.np_, bary, wq, _ref(0.0), 2, 1)
    with pytest.raises(ValueError):
        oracle.Oracle(sc.with_(dudn=1, src_c0=0.0)).adjoint_grad(code, bary, wq, _ref(0.0), 2, 1)
    g, lam, uoff, st = o.adjoint_grad(code[:0], bary[:0], wq[:0], _ref(0.0), 2, 1)
    assert g[0] == 0 and lam.size == 0
