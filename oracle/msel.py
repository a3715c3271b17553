"""FP64 oracle of the learned m-selector (numpy, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The selector is not part of the paper; its pieces are defined from the paper's
estimator and from textbook definitions:

* ``expected_e2`` -- expected squared Frobenius error of the covariance
  estimator C_n (Sec. V) relative to ||C_emp||_F^2, the expectation taken over
  the sampling only.  Each entry of C_n is (1/n) sum_i of independent
  per-sample terms; a coordinate is kept with probability m/p (Lemma in
  App. B) and a pair with probability m(m-1)/(p(p-1)) (Thm. in App. B), and
  the rescaling makes every term unbiased, so the variance of a term is its
  square times (1/q - 1).  Pinned by enumerating every m-subset for tiny
  (p, m) and n = 1, 2 with the literal estimator of ``oracle_def``.
* ``label_m`` -- smallest m in [2, p] with expected_e2 <= t^2 (a scan over m).
  Pinned through ``expected_e2`` and by the scan being the definition.
* ``features`` -- the 32 block statistics (layout in ``FEATURE_NAMES``).
  Pinned: quantiles against ``numpy.quantile(method="lower")``; the pair
  statistic against a brute-force double loop over rows; the plug-in label
  against ``label_m`` when the subset is the whole block.
* ``mlp_*`` -- the 32-64-64-1 ReLU network, the expectile loss, its gradient
  and Adam; pinned by central finite differences and by ``torch.autograd`` /
  ``torch.optim.Adam`` on the CPU in FP64.  ``bf16_round`` is pinned against
  torch's float32 -> bfloat16 conversion.
"""
import numpy as np

from . import ref

QUANT_PER_MILLE = (50, 150, 300, 500, 700, 850, 950, 1000)
N_FEAT = 32
N_IN, N_H = 32, 64
OFF_W1, OFF_B1 = 0, 2048
OFF_W2, OFF_B2 = 2112, 6208
OFF_W3, OFF_B3 = 6272, 6336
N_PARAMS = 6337


def row_moments(X):
    """(sum_j x_ij^2, sum_j x_ij^4, max_j x_ij^2) per row, FP64."""
    X = np.asarray(X, dtype=np.float64)
    sq = X * X
    return np.stack([sq.sum(1), (sq * sq).sum(1), sq.max(1)], axis=1)


def frob_diff(A, B):
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    return float(((A - B) ** 2).sum()), float((B * B).sum())


def transform(X, D):
    """y_i = H D x_i for each row (Sec. III, eq. ROS), FP64."""
    Y = np.asarray(X, dtype=np.float64) * np.asarray(D, dtype=np.float64)[None, :]
    return np.stack([ref.fwht_normalized(row) for row in Y]) if len(Y) else Y


def _second_moments(Y):
    """M[j][k] = sum_i y_ij^2 y_ik^2."""
    S = Y * Y
    return S.T @ S


def expected_e2(Y, m, C_fro2=None, M=None):
    """E||C_n - C_emp||_F^2 / ||C_emp||_F^2 over the sampling (Sec. V; App. B)."""
    Y = np.asarray(Y, dtype=np.float64)
    n, p = Y.shape
    if M is None:
        M = _second_moments(Y)
    if C_fro2 is None:
        C = Y.T @ Y / n
        C_fro2 = float((C * C).sum())
    q1 = m / p
    q2 = m * (m - 1) / (p * (p - 1))
    diag = float(np.trace(M))
    off = float(M.sum()) - diag
    return ((1.0 / q2 - 1.0) * off + (1.0 / q1 - 1.0) * diag) / (n * n * C_fro2)


def label_m(Y, t):
    """Smallest m in [2, p] whose expected squared relative error is <= t^2."""
    Y = np.asarray(Y, dtype=np.float64)
    n, p = Y.shape
    C = Y.T @ Y / n
    F2 = float((C * C).sum())
    if not F2 > 0.0:
        return 2
    M = _second_moments(Y)
    for m in range(2, p + 1):
        if expected_e2(Y, m, F2, M) <= t * t:
            return m
    return p


def _rule_from_moments(p, n, A, B, F2, t):
    """The label scan with the moments given directly (used by feature 31)."""
    if not F2 > 0.0:
        return p
    for m in range(2, p + 1):
        q1 = m / p
        q2 = m * (m - 1) / (p * (p - 1))
        if ((1.0 / q2 - 1.0) * A + (1.0 / q1 - 1.0) * B) / (n * n * F2) <= t * t:
            return m
    return p


def quantile_lower(v, q_per_mille):
    v = np.sort(np.asarray(v, dtype=np.float64))
    return v[(q_per_mille * (len(v) - 1)) // 1000]


def features(Xsub, D, n, t):
    """32 features of a block of n rows from its first rows Xsub (2 <= s <= 1024)."""
    Xsub = np.asarray(Xsub, dtype=np.float64)
    s, p = Xsub.shape
    Y = transform(Xsub, D)
    s2r = (Xsub * Xsub).sum(1)
    s4r = (Xsub ** 4).sum(1)
    mxr = (Xsub * Xsub).max(1)
    s2y = (Y * Y).sum(1)
    s4y = (Y ** 4).sum(1)
    mxy = (Y * Y).max(1)
    with np.errstate(divide="ignore", invalid="ignore"):
        coh_r = np.where(s2r > 0, np.log(p * mxr / np.where(s2r > 0, s2r, 1.0)), 0.0)
        coh_y = np.where(s2y > 0, np.log(p * mxy / np.where(s2y > 0, s2y, 1.0)), 0.0)
        flat_r = np.where(s2r > 0, p * s4r / np.where(s2r > 0, s2r, 1.0) ** 2, 1.0)
        flat_y = np.where(s2y > 0, p * s4y / np.where(s2y > 0, s2y, 1.0) ** 2, 1.0)
    mean_r = s2r.mean()
    mean_y = s2y.mean()
    C = Y.T @ Y / s
    F2s = float((C * C).sum())
    U = (s * s * F2s - (s2y * s2y).sum()) / (s * (s - 1))
    f = np.zeros(N_FEAT)
    with np.errstate(divide="ignore", invalid="ignore"):
        f[0] = np.log(mean_r)
        for k, q in enumerate(QUANT_PER_MILLE):
            f[1 + k] = quantile_lower(s2r, q) / mean_r
            f[9 + k] = quantile_lower(coh_r, q)
            f[17 + k] = quantile_lower(coh_y, q)
        f[25] = np.log(flat_y.mean())
        f[26] = np.log(flat_r.mean())
        f[27] = np.log(max(U, 1e-300) / mean_y ** 2)
        f[28] = np.log(F2s / mean_y ** 2)
    f[29] = np.log(n)
    f[30] = np.log(p)
    F2n = (s2y * s2y).mean() / n + (n - 1) / n * U
    A = n * (s2y * s2y - s4y).mean()
    B = n * s4y.mean()
    f[31] = np.log(_rule_from_moments(p, n, A, B, F2n, t) / p)
    return f


FEATURE_NAMES = (
    ["log_mean_sq_norm"] + [f"norm_q{q}" for q in QUANT_PER_MILLE] + [f"raw_coh_q{q}" for q in QUANT_PER_MILLE]
    + [f"pre_coh_q{q}" for q in QUANT_PER_MILLE]
    + ["log_flat_pre", "log_flat_raw", "log_pair_stat", "log_sub_fro", "log_n", "log_p", "log_plugin_gamma"])


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    return (P[OFF_W1:OFF_B1].reshape(N_H, N_IN), P[OFF_B1:OFF_W2], P[OFF_W2:OFF_B2].reshape(N_H, N_H),
            P[OFF_B2:OFF_W3], P[OFF_W3:OFF_B3], P[OFF_B3])


def mlp_forward(P, F, mu, sd):
    """Output and activations (xn, h1, h2) of the network, FP64."""
    W1, b1, W2, b2, w3, b3 = unpack(P)
    xn = (np.asarray(F, np.float64) - np.asarray(mu, np.float64)) / np.asarray(sd, np.float64)
    h1 = np.maximum(xn @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ w3 + b3, (xn, h1, h2)


def expectile_loss(pred, target, tau):
    r = np.asarray(target, np.float64) - np.asarray(pred, np.float64)
    w = np.where(r < 0, 1.0 - tau, tau)
    return float((w * r * r).mean())


def mlp_grad(P, F, mu, sd, target, tau):
    """Gradient of the expectile loss with respect to the packed parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(P)
    y, (xn, h1, h2) = mlp_forward(P, F, mu, sd)
    B = len(y)
    r = np.asarray(target, np.float64) - y
    w = np.where(r < 0, 1.0 - tau, tau)
    gy = -2.0 * w * r / B
    g = np.zeros(N_PARAMS)
    g[OFF_B3] = gy.sum()
    g[OFF_W3:OFF_B3] = gy @ h2
    d2 = np.outer(gy, w3) * (h2 > 0)
    g[OFF_W2:OFF_B2] = (d2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = d2.sum(0)
    d1 = (d2 @ W2) * (h1 > 0)
    g[OFF_W1:OFF_B1] = (d1.T @ xn).ravel()
    g[OFF_B1:OFF_W2] = d1.sum(0)
    return g, expectile_loss(y, target, tau)


def adam_step(P, g, m1, m2, step, lr, b1, b2, eps):
    """One Adam update (Kingma & Ba); returns new (P, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mhat = m1 / (1 - b1 ** step)
    vhat = m2 / (1 - b2 ** step)
    return P - lr * mhat / (np.sqrt(vhat) + eps), m1, m2


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def mlp_predict_bf16(P, F, mu, sd, gmin, gmax, fallback):
    """Inference with BF16 weights, BF16 standardized inputs and first hidden
    layer, exact (FP64) sums; gamma = clamp(exp(y)) or the fallback."""
    Pb = bf16_round(np.asarray(P, np.float32)).astype(np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(Pb)
    F = np.asarray(F, np.float64)
    # rows with non-finite features propagate NaN and take the fallback below
    with np.errstate(over="ignore", invalid="ignore"):
        xn = ((F.astype(np.float32) - np.asarray(mu, np.float32)) / np.asarray(sd, np.float32))
        xn = bf16_round(xn).astype(np.float64)
        h1 = np.maximum(xn @ W1.T + b1, 0.0)
        h1 = bf16_round(h1.astype(np.float32)).astype(np.float64)
        h2 = np.maximum(h1 @ W2.T + b2, 0.0)
        y = h2 @ w3 + b3
        g = np.exp(y)
    bad = ~np.isfinite(F).all(1) | ~np.isfinite(g)
    g = np.where(bad, fallback, g)
    return np.clip(g, gmin, gmax), y
