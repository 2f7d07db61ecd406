"""Ablations of Sec. 6.3 on the oracle (CPU), restated as tests.

* The backward difference of eq. (dudn_fd_estimate) at offset delta: on the
  screened disk with g = 1 the radial symmetry makes the differential
  walk's expectation exact, u(x) (1 - u(R - delta)) / delta in place of
  u(x) du/dr(R), so the estimator's bias has a closed form at every delta;
  the oracle's mean follows it through a halving sweep of (eps, delta), and
  the bias falls about linearly with delta.
* The product estimators of Sec. 5.3 for the squared loss
  L = 1/2 sum_p (u_p - uref_p)^2: the correlated product (u and udot from
  the same walks) is biased by the per-walk covariance over W; the
  uncorrelated product (independent walks for u) and the U-statistic of
  eq. (ustatistics) are unbiased; their RMSEs are compared at equal walks.
"""
import math

import numpy as np
import pytest
from scipy import special

import scenes


def test_backward_difference_bias_halves_with_delta(oracle_mod):
    sigma = 10.0
    k = math.sqrt(sigma)
    u = lambda r: special.i0(k * r) / special.i0(k)
    dudr = k * special.i1(k) / special.i0(k)
    X = np.array([[0.2, 0.1], [-0.3, 0.25]])
    ux = u(np.hypot(X[:, 0], X[:, 1]))
    biases = []
    for delta in (0.2, 0.1, 0.05):
        sc = scenes.c1_polygon(512, g="one", eps=1e-4, delta=delta, sigma=sigma)
        jm, jv, _, _ = oracle_mod.Oracle(sc).jvp(X, 65536, 17)
        est = jm[:, 0]
        se = np.sqrt(jv[:, 0])
        # dv/dR = v/R: V_n = 1 and du/dR = -u(x) du/dr(R); the estimator
        # replaces du/dr(R) by the backward difference (1 - u(R - delta))/delta
        expect = -ux * (1 - u(1 - delta)) / delta
        assert np.all(np.abs(est - expect) <= 4 * se + 2e-3 * np.abs(expect)), (delta, est, expect, se)
        biases.append(float(np.mean(est + ux * dudr)))
    # the bias is positive (the difference underestimates the slope of a
    # convex u) and about halves with delta
    assert biases[0] > biases[1] > biases[2] > 0
    for a, b in zip(biases, biases[1:]):
        assert 1.6 < a / b < 2.2, biases


def test_product_estimators_of_the_squared_loss(oracle_mod):
    """Sec. 5.3 on a 256-segment star: bias and RMSE of the three estimators
    of dL/dpi at W = 8 walks per point, over 150 replicates, against a
    reference from the unbiased forms at many walks."""
    sc = scenes.c2_star(n=256, kmax=4, eps=2e-3, delta=2e-2)
    X = scenes.star_points(8, 41)
    uref = np.full(len(X), 0.2)
    o = oracle_mod.Oracle(sc)
    # reference: u and udot means from independent walks at many walks
    um, _, _ = o.solve(X, 32768, 42)
    ud, _, _, _ = o.jvp(X, 32768, 43)
    gstar = ((um - uref)[:, None] * ud).sum(0)
    W, R = 8, 150
    corr, unc, ust = [], [], []
    for r in range(R):
        rec = o.walk_records(X, W, 1000 + r, mode=1)
        uj, udw = rec["u"], rec["udot"]               # (P, W), (P, W, N)
        ubar = uj.mean(1)
        udbar = udw.mean(1)
        corr.append(((ubar - uref)[:, None] * udbar).sum(0))
        uf, _, _ = o.solve(X, W, 5000 + r)             # independent forward walks
        unc.append(((uf - uref)[:, None] * udbar).sum(0))
        # U-statistic: pairs i != j of the same walks
        S_u = uj.sum(1)
        S_ud = udw.sum(1)
        pair = (S_u[:, None] * S_ud - (uj[:, :, None] * udw).sum(1)) / (W * (W - 1))
        ust.append((pair - uref[:, None] * udbar).sum(0))
    corr, unc, ust = (np.array(a) for a in (corr, unc, ust))
    se = lambda a: a.std(0, ddof=1) / math.sqrt(R)
    # the unbiased forms agree with the reference
    for name, a in (("uncorrelated", unc), ("U-statistic", ust)):
        z = (a.mean(0) - gstar) / np.sqrt(se(a) ** 2 + 1e-12)
        assert np.mean(z ** 2) < 2.0 and np.abs(z).max() < 4.5, (name, z)
    # the correlated product's bias is the per-walk covariance of u and
    # udot over W (summed over points), estimated from long records
    rec = o.walk_records(X, 4096, 77, mode=1)
    cov = ((rec["u"] - rec["u"].mean(1, keepdims=True))[:, :, None] *
           (rec["udot"] - rec["udot"].mean(1, keepdims=True))).sum(1) / (4096 - 1)
    pred = cov.sum(0) / W
    z = (corr.mean(0) - gstar - pred) / np.sqrt(se(corr) ** 2 + 1e-12)
    assert np.mean(z ** 2) < 2.5, z
    rmse = lambda a: float(np.sqrt(np.mean((a - gstar) ** 2)))
    print(f"RMSE at W = {W}: correlated {rmse(corr):.4g}, uncorrelated {rmse(unc):.4g}, "
          f"U-statistic {rmse(ust):.4g}")
