"""Bound calculators from the paper's theorems (TEST INFRASTRUCTURE ONLY).

Used by the statistical tests; pinned by the worked values the paper prints
(Cor. "sampleMean": 137.2 / 15.1 / 1.6, golden fixture ``tests/golden``).
``mean_error_t`` and ``cov_error_t`` are checked against the oracle's
estimators at the setups of the theorems' figures (errors below the bounds and
of the order the figures show).
Logarithms are natural: the printed values reproduce only with ln.
"""
import math


def tau(m, p):
    """eq. tau-m-p: max(p/m - 1, 1)."""
    return max(p / m - 1.0, 1.0)


def mean_error_t(delta1, n, m, p, x_max, x_max_row):
    """Thm. sampleMean, second remark: the l_inf error t that holds with
    probability 1 - delta1 (solving eq. fail_prob_sample_mean for t)."""
    L = math.log(2.0 * p / delta1)
    a = tau(m, p) / 3.0 * x_max * L
    return (a + math.sqrt(a * a + 2.0 * (p / m - 1.0) * L * x_max_row ** 2)) / n


def cor5_m_lower_bound(n, p, t, eta=1.0):
    """Cor. sampleMean, eq. lower-bound-m."""
    return (1.0 / n) * (4.0 / eta) * math.log(200.0 * n * p) * math.log(2000.0 * p) * (
        t ** -2 + math.sqrt(p) / (3.0 * t))


def delta3(t, nk, m, p):
    """Thm. RRT, eq. delta3: failure probability of ||H_k - I||_2 <= t."""
    return p * math.exp(-nk * t * t / 2.0 / ((p / m - 1.0) + (p / m + 1.0) * t / 3.0))


def t_for_delta3(delta, nk, m, p):
    """Inverse of delta3 in t (monotone decreasing), by bisection."""
    lo, hi = 0.0, 1e6
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if delta3(mid, nk, m, p) > delta:
            lo = mid
        else:
            hi = mid
    return hi


def cor_rho_norm_bound(m, p, alpha, n=1, eta=1.0):
    """Cor. cor-rho: ||w_i||^2 <= (m/p)(2/eta) log(2np/alpha) ||x_i||^2."""
    return (m / p) * (2.0 / eta) * math.log(2.0 * n * p / alpha)


def thm1_tail(t, eta=1.0):
    """Thm. FJLT: P(|y_j| >= t ||x|| / sqrt(p)) <= 2 exp(-eta t^2 / 2)."""
    return 2.0 * math.exp(-eta * t * t / 2.0)


def cov_error_t(delta2, X, m, rho=1.0):
    """Thm. covariance: the spectral-norm error t of C_n that holds with
    probability 1 - delta2, solving eq. cov-converge-delta2 for t with L from
    eq. covariance-L and sigma^2 at its upper bound eq. covariance_sigma.  The
    samples are the rows of X here (the paper's X is p x n): ||X||_maxCol is
    the largest sample norm, max_j sum_i X_ji^4 runs over coordinates."""
    import numpy as np

    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    maxcol2 = float(np.max(np.sum(X * X, axis=1)))
    xmax2 = float(np.max(np.abs(X))) ** 2
    C = X.T @ X / n
    a = p * (p - 1) / (m * (m - 1))
    b = p * (p - 1) * (p - m) / (m * (m - 1) ** 2)
    L = ((a * rho + 1.0) * maxcol2 + p * (p - m) / (m * (m - 1)) * xmax2) / n
    sigma2 = ((a * rho - 1.0) * maxcol2 * float(np.linalg.norm(C, 2))
              + b * rho * maxcol2 * float(np.max(np.diag(C)))
              + 2.0 * b * xmax2 * float(np.sum(X * X)) / n
              + p * (p - m) ** 2 / (m * (m - 1) ** 2) * float(np.max(np.sum(X ** 4, axis=0))) / n) / n
    ell = math.log(p / delta2)
    return ell * L / 3.0 + math.sqrt((ell * L / 3.0) ** 2 + 2.0 * ell * sigma2)
