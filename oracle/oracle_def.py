"""Literal-matrix oracle for tiny sizes (TEST INFRASTRUCTURE ONLY).

Everything here is the paper's algebra typed in with explicit matrices
(arXiv 1511.00152): an explicit normalized Hadamard matrix from
``scipy.linalg.hadamard``, an explicit diagonal D, explicit p x m sampling
matrices R_i whose columns are canonical basis vectors, and the estimators as
displayed.  Samples are the columns of X here, as in the paper.

The random choices the paper leaves open are drawn from numpy's own
Philox4x64-10 bit generator, so this file shares no random-number code with
the C oracle: word streams, Lemire's method and Floyd's algorithm are
re-expressed here in plain Python integers.
"""
import math

import numpy as np
import scipy.linalg

MASK64 = (1 << 64) - 1


# --------------------------------------------------------------------------
# Random words: numpy.random.Philox advances its 256-bit counter before it
# produces a block, so the block for counter c is what a generator whose
# counter is set to c - 1 returns first.
# --------------------------------------------------------------------------
def philox_block(counter, key):
    c = 0
    for w in reversed([int(x) for x in counter]):
        c = (c << 64) | (w & MASK64)
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * k)) & MASK64 for k in range(4)], dtype=np.uint64)
    g = np.random.Philox(key=np.array([int(key[0]), int(key[1])], dtype=np.uint64), counter=words)
    return [int(v) for v in g.random_raw(4)]


def word_stream(seed, c1, c2):
    """32-bit words of blocks (b, c1, c2, 0), b = 0, 1, ...; low half first."""
    b = 0
    while True:
        for w in philox_block([b, c1, c2, 0], [seed, 0]):
            yield w & 0xFFFFFFFF
            yield w >> 32
        b += 1


def lemire(rng, words):
    """Uniform integer in [0, rng) from 32-bit words (Lemire 2019)."""
    x = next(words)
    prod = x * rng
    low = prod & 0xFFFFFFFF
    if low < rng:
        thresh = (2 ** 32 - rng) % rng
        while low < thresh:
            x = next(words)
            prod = x * rng
            low = prod & 0xFFFFFFFF
    return prod >> 32


def kept_set(seed, i, p, m):
    """Floyd: for t = p-m..p-1 draw r in {0..t}; add r, or t if r is taken."""
    words = word_stream(seed, i, 0)
    S = set()
    for t in range(p - m, p):
        r = lemire(t + 1, words)
        S.add(t if r in S else r)
    return sorted(S)


def signs(seed, p):
    """D_j from bit j mod 64 of word (j div 64) mod 4 of block (j div 256, 0, 1, 0)."""
    D = np.empty(p)
    for j in range(p):
        w = philox_block([j // 256, 0, 1, 0], [seed, 0])[(j // 64) % 4]
        D[j] = -1.0 if (w >> (j % 64)) & 1 else 1.0
    return D


# --------------------------------------------------------------------------
# Sec. III: the ROS y = H D x with explicit matrices.
# --------------------------------------------------------------------------
def hadamard(p):
    return scipy.linalg.hadamard(p).astype(np.float64) / math.sqrt(p)


def ros_matrix(seed, p):
    return hadamard(p) @ np.diag(signs(seed, p))


def sampling_matrix(idx, p):
    """R in R^{p x m}: columns are the canonical basis vectors e_idx."""
    R = np.zeros((p, len(idx)))
    for c, j in enumerate(idx):
        R[j, c] = 1.0
    return R


def compress(X, seed, m):
    """X is p x n (samples are columns).  Returns (Y, W, idx list)
    with Y = H D X and w_i = R_i R_i^T y_i."""
    p, n = X.shape
    Y = ros_matrix(seed, p) @ X
    W = np.zeros_like(Y)
    idx = []
    for i in range(n):
        ix = kept_set(seed, i, p, m)
        R = sampling_matrix(ix, p)
        W[:, i] = R @ R.T @ Y[:, i]
        idx.append(ix)
    return Y, W, idx


# --------------------------------------------------------------------------
# Sec. V: covariance estimators, as displayed.
# --------------------------------------------------------------------------
def cov_emp_hat(Y, idx, m):
    p, n = Y.shape
    acc = np.zeros((p, p))
    for i in range(n):
        R = sampling_matrix(idx[i], p)
        y = Y[:, i:i + 1]
        acc += R @ R.T @ y @ y.T @ R @ R.T
    return (p * (p - 1)) / (m * (m - 1)) * acc / n


def cov_n(Y, idx, m):
    p = Y.shape[0]
    Ce = cov_emp_hat(Y, idx, m)
    return Ce - (p - m) / (p - 1) * np.diag(np.diag(Ce))


def cov_emp(Y):
    return Y @ Y.T / Y.shape[1]


def mean_hat(Y, idx, m):
    """Thm. sampleMean: (p/m)(1/n) sum_i R_i R_i^T y_i."""
    p, n = Y.shape
    acc = np.zeros(p)
    for i in range(n):
        R = sampling_matrix(idx[i], p)
        acc += R @ R.T @ Y[:, i]
    return p / m * acc / n


# --------------------------------------------------------------------------
# Sec. VI: sparsified K-means, one assignment + update round, with R_i.
# centers: p x K matrix mu' (columns are centers).
# --------------------------------------------------------------------------
def kmeans_step(Y, idx, centers):
    p, n = Y.shape
    K = centers.shape[1]
    assign = np.zeros(n, dtype=np.int64)
    obj = 0.0
    for i in range(n):
        R = sampling_matrix(idx[i], p)
        z = R.T @ Y[:, i]
        d = [float(np.sum((z - R.T @ centers[:, k]) ** 2)) for k in range(K)]
        assign[i] = int(np.argmin(d))  # first minimum on ties
        obj += d[assign[i]]
    new = centers.copy()
    for k in range(K):
        lhs = np.zeros((p, p))
        rhs = np.zeros(p)
        for i in np.nonzero(assign == k)[0]:
            R = sampling_matrix(idx[i], p)
            lhs += R @ R.T
            rhs += R @ R.T @ Y[:, i]
        # eq. mu_update_one: the left-hand matrix is diagonal (the counts
        # n_k^(j)); rows with a zero count cannot be estimated and keep mu'.
        counts = np.diag(lhs)
        ok = counts > 0
        new[ok, k] = rhs[ok] / counts[ok]
    return new, assign, obj


def unmix(seed, centers):
    """eq. mu-mu': mu = (H D)^T mu'."""
    p = centers.shape[0]
    return ros_matrix(seed, p).T @ centers


def lloyd_step(X, centers):
    """Standard K-means (Sec. VI, steps 1 and 2) on full samples (columns)."""
    p, n = X.shape
    K = centers.shape[1]
    d = np.array([[np.sum((X[:, i] - centers[:, k]) ** 2) for k in range(K)] for i in range(n)])
    assign = np.argmin(d, axis=1)
    new = centers.copy()
    for k in range(K):
        sel = assign == k
        if sel.any():
            new[:, k] = X[:, sel].mean(axis=1)
    return new, assign, float(d[np.arange(n), assign].sum())
