"""Statistical checks of a sample against the standard normal law.

TEST INFRASTRUCTURE ONLY.  Used on oracle output (to pin the oracle to the
mathematics) and on GPU output (as a property that holds at any size).
Reference law: Phi(x) = erfc(-x/sqrt 2)/2.  Standard errors of the sample
moments of N(0,1): mean 1/sqrt(n), variance sqrt(2/n), skewness sqrt(6/n),
excess kurtosis sqrt(24/n).
"""
import math

import numpy as np
from scipy import special


def moments(x):
    """Mean, variance, skewness, excess kurtosis (float64 accumulation) and
    their standard errors under N(0,1)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    m1 = float(np.mean(x))
    c = x - m1
    m2 = float(np.mean(c * c))
    m3 = float(np.mean(c * c * c))
    m4 = float(np.mean((c * c) * (c * c)))
    skew = m3 / m2 ** 1.5
    kurt = m4 / (m2 * m2) - 3.0
    se = dict(mean=1 / math.sqrt(n), var=math.sqrt(2 / n), skew=math.sqrt(6 / n),
              kurt=math.sqrt(24 / n))
    return dict(n=n, mean=m1, var=m2, skew=skew, kurt=kurt, se=se)


def moment_zscores(x):
    m = moments(x)
    se = m["se"]
    return dict(mean=m["mean"] / se["mean"], var=(m["var"] - 1) / se["var"],
                skew=m["skew"] / se["skew"], kurt=m["kurt"] / se["kurt"])


def phi(x):
    return 0.5 * special.erfc(-np.asarray(x, dtype=np.float64) / math.sqrt(2.0))


def ks_statistic(x, cdf=phi):
    """Two-sided Kolmogorov-Smirnov distance between the sample and cdf."""
    xs = np.sort(np.asarray(x, dtype=np.float64))
    n = xs.size
    F = cdf(xs)
    i = np.arange(1, n + 1, dtype=np.float64)
    d_plus = np.max(i / n - F)
    d_minus = np.max(F - (i - 1) / n)
    return float(max(d_plus, d_minus))


def ks_critical(n, alpha=0.01):
    """Asymptotic KS critical value sqrt(-ln(alpha/2)/2)/sqrt(n)."""
    return math.sqrt(-math.log(alpha / 2) / 2) / math.sqrt(n)


def tail_count_z(x, r):
    """z-score of the count of |x| > r against n erfc(r/sqrt 2) (binomial)."""
    x = np.asarray(x)
    n = x.size
    p = math.erfc(r / math.sqrt(2.0))
    k = int(np.count_nonzero(np.abs(x) > r))
    return (k - n * p) / math.sqrt(n * p * (1 - p)), k, n * p


def tail_conditional_cdf(r):
    """P(|X| <= x given |X| > r) for the standard normal, x > r."""
    er = special.erfc(r / math.sqrt(2.0))

    def F(x):
        return (er - special.erfc(np.asarray(x) / math.sqrt(2.0))) / er
    return F
