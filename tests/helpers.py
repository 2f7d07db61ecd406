"""Statistical comparison rules shared by the tests (no estimator arithmetic)."""
import math

import numpy as np


def check_vs_exact(est, se, exact, budget, name="", frac=0.01):
    """Monte Carlo estimates against a closed form.

    Per point: |est - exact| <= 3 se + budget, allowing a fraction ``frac`` of
    points (plus one) to exceed it.  Aggregate: the mean error over points is
    within 4 standard errors of the mean plus the bias budget.
    """
    est, se, exact = (np.asarray(a, float).ravel() for a in (est, se, exact))
    err = est - exact
    bad = np.abs(err) > 3 * se + budget
    nbad = int(bad.sum())
    allowed = 1 + int(frac * err.size)
    msg = (f"{name}: {nbad}/{err.size} points beyond 3SE+{budget:g}; "
           f"max|err|={np.abs(err).max():.3g} mean err={err.mean():.3g} "
           f"mean SE={se.mean():.3g}")
    assert nbad <= allowed, msg
    se_mean = math.sqrt(float((se ** 2).sum())) / err.size
    assert abs(err.mean()) <= 4 * se_mean + budget, msg + f" (SE of mean {se_mean:.3g})"
    return msg


def parity(a, se_a, b, se_b, abs_tol=1e-4, name=""):
    """GPU-vs-oracle statistical parity rule.

    Per point z = (a - b)/sqrt(se_a^2 + se_b^2).  Pass if at most 1% of points
    (plus one) differ by more than 3 SE + abs_tol, and mean z^2 lies within
    1 +- 5 sqrt(2/P)."""
    a, se_a, b, se_b = (np.asarray(x, float).ravel() for x in (a, se_a, b, se_b))
    se = np.sqrt(se_a ** 2 + se_b ** 2)
    d = a - b
    bad = np.abs(d) > 3 * se + abs_tol
    P = d.size
    nbad = int(bad.sum())
    ok = se > 0
    z2 = float(np.mean((d[ok] / se[ok]) ** 2)) if ok.any() else 0.0
    lim = 5 * math.sqrt(2.0 / max(1, ok.sum()))
    msg = (f"{name}: {nbad}/{P} beyond 3SE+{abs_tol:g}, mean z^2={z2:.3f} "
           f"(allowed 1+-{lim:.3f}), max|d|={np.abs(d).max():.3g}")
    assert nbad <= 1 + int(0.01 * P), msg
    if ok.sum() >= 8:
        assert abs(z2 - 1.0) <= lim, msg
    return msg
