"""Statistical acceptance criteria shared by the estimator tests.

A Monte Carlo estimate is compared with a reference value through per-point
z-scores z_i = (m_i - u_i) / se_i.  Even an exact estimator exceeds |z| > 3 at
a fraction of points, so the acceptance test is on the population of z-scores:

* the count of |z| > 3 must not exceed the 1e-6 upper quantile of a binomial
  with the two-sided tail probability of a Student t with (n_walks - 1) degrees
  of freedom (the SE is itself estimated from the walks);
* the mean z must lie within 5 / sqrt(N) of zero (plus an optional bias slack);
* the variance of z must lie in a band around the t variance.
"""
import numpy as np
from scipy import stats


def zscore_check(mean, se, ref, n_walks, bias_slack=0.0, var_band=(0.75, 1.35), label="", allow=None,
                 skewed=False):
    """``allow`` is an optional per-point bias allowance (e.g. the epsilon-shell
    bias eps |grad u|): deviations are shrunk by it before dividing by se.

    ``skewed``: for walk values with long one-sided tails (rare long
    excursions, the Green's function singularity of boundary walkers) the
    sample SE of a point is correlated with its deviation, and the mean of
    the per-point z is not centred even for an unbiased estimator.  Then
    unbiasedness is checked on the mean deviation itself (within 5 of its
    standard errors plus the mean allowance), and the variance band on z
    before the allowance; the exceedance count is checked as always."""
    mean = np.asarray(mean, float)
    se = np.asarray(se, float)
    ref = np.asarray(ref, float)
    ok = se > 0
    dev = mean[ok] - ref[ok]
    if allow is not None:
        a = np.broadcast_to(np.asarray(allow, float), mean.shape)[ok]
        dev = np.sign(dev) * np.maximum(np.abs(dev) - a, 0.0)
    z = dev / se[ok]
    N = z.size
    dof = max(int(np.min(n_walks)) - 1, 3)
    p3 = 2.0 * stats.t.sf(3.0, dof)
    limit = stats.binom.ppf(1.0 - 1e-6, N, p3)
    n_exceed = int(np.sum(np.abs(z) > 3.0))
    tvar = dof / (dof - 2.0)
    info = dict(N=N, mean_z=float(z.mean()), var_z=float(z.var()), n_exceed=n_exceed,
                limit=float(limit), max_abs_z=float(np.abs(z).max()) if N else 0.0, label=label)
    assert n_exceed <= limit, info
    if skewed:
        raw = mean[ok] - ref[ok]
        zr = raw / se[ok]
        tol = 5.0 * np.sqrt(np.sum(se[ok] ** 2)) / N
        if allow is not None:
            tol += float(np.mean(np.broadcast_to(np.asarray(allow, float), mean.shape)[ok]))
        info.update(mean_dev=float(raw.mean()), mean_dev_tol=float(tol), var_z_raw=float(zr.var()))
        assert abs(raw.mean()) <= tol, info
        assert var_band[0] <= zr.var() / tvar <= var_band[1], info
        return info
    assert abs(z.mean()) <= 5.0 / np.sqrt(N) + bias_slack, info
    assert var_band[0] <= z.var() / tvar <= var_band[1], info
    return info


def two_sample_z(m1, se1, m2, se2):
    s = np.sqrt(np.asarray(se1) ** 2 + np.asarray(se2) ** 2)
    return (np.asarray(m1) - np.asarray(m2)) / s
