"""ctypes wrapper over the C oracle ``liboracle.so`` (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Functions and the passages they follow (paper = arXiv 1511.00152):

* ``philox4x64_10`` -- block function of Philox4x64-10 (Salmon et al., SC'11);
  pinned bit-exactly to ``numpy.random.Philox``.
* ``lemire_from_words`` -- Lemire's multiply-and-reject uniform integer; pinned
  by exhaustive enumeration at 8-bit word width.
* ``floyd_from_draws`` / ``sample_indices`` -- exact-m sampling without
  replacement (Sec. I setup; App. B); pinned by enumerating every draw sequence
  at tiny (p, m), by inclusion frequencies m/p (Lemma in App. B) and pair
  frequencies m(m-1)/(p(p-1)) (Thm. in App. B), and against ``oracle_def``
  which draws with numpy's own Philox.
* ``signs`` -- the random diagonal D (Sec. III, eq. ROS); pinned against
  ``oracle_def`` (numpy Philox) and E[D]=0 statistics.
* ``fwht_normalized`` -- y = H x with H the normalized Sylvester Hadamard
  matrix (Sec. III); pinned against ``scipy.linalg.hadamard``.
* ``compress`` -- Alg. 1 first loop; pinned against ``oracle_def`` and norm
  preservation.
* ``gram_accumulate`` / ``cov_finalize`` -- Sec. V estimators; pinned by exact
  enumeration of all m-subsets (unbiasedness, App. C expectations), by the
  m = p special case, and against ``oracle_def``.
* ``kmeans_step`` / ``unmix`` / ``kmeanspp`` -- Sec. VI and Alg. 1; pinned by
  the m = p reduction to Lloyd's algorithm (scikit-learn and a brute-force
  loop), monotone objective, and ``oracle_def``.  The seeding follows Arthur &
  Vassilvitskii with the sparsified distance of Sec. VI; it is pinned by its
  sampling law (first center uniform, the next one with probability D^2 / sum
  D^2), checked by Monte Carlo over seeds; which stream words it consumes is
  a reading (starting point r reads counter (b, r, 2, 0), pinned against
  numpy's Philox).
* ``sparsified_kmeans_best`` -- best of R starting points (Sec. VII runs):
  the kept start is the argmin of the final objectives recomputed by a
  direct numpy sum over each start's own assignment.
* ``y_entry`` -- one entry of H D x from the definition (row of H times D x).
* ``mean_estimate`` -- Thm. "sampleMean"; pinned by enumeration (unbiased).
* ``dct_orthonormal`` / ``compress_dct`` / ``unmix_dct`` -- the DCT form of the
  preconditioner (Sec. III; Thm. 1 with eta = 1/2) for p not a power of two;
  pinned against the DCT-II matrix written from its definition, the inverse
  round trip at m = p, and Thm. 1's tail with eta = 1/2 by Monte Carlo.
* ``clustering_accuracy`` -- Sec. VII's accuracy against ground-truth labels;
  pinned by brute force over every matching at small K.
* ``principal_components`` / ``explained_variance`` -- PCA on the covariance
  estimate (Sec. V) and the fraction of explained variance used in the
  column-sampling comparison (Sec. II); pinned by the canonical-subset closed
  form, the full-basis value 1, rotation invariance within the span, and the
  Ky Fan value (top-k singular values of X from an independent SVD).
* ``kmeans_2pass`` -- Alg. "Sparsified K-means, 2-pass": one pass over the
  original rows after the one-pass run; pinned against per-label means
  (``numpy.add.at``) and nearest centers (``scipy.spatial.distance.cdist``),
  by the Lloyd fixed point (converged assignments and centers come back
  unchanged) and by the empty-cluster rule.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        u64 = ctypes.c_uint64
        i32 = ctypes.c_int
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_lemire_from_words.argtypes = [ctypes.c_uint32, i32, P, i32, P]
        L.orc_lemire_from_words.restype = ctypes.c_uint32
        L.orc_floyd_from_draws.argtypes = [i64, i64, P, P]
        L.orc_floyd_from_draws.restype = i32
        L.orc_sample_indices.argtypes = [u64, u64, i64, i64, P]
        L.orc_signs.argtypes = [u64, i64, P]
        L.orc_fwht_normalized.argtypes = [P, i64]
        L.orc_y_entry_f64.argtypes = [P, i64, i64, P]
        L.orc_y_entry_f64.restype = ctypes.c_double
        L.orc_y_entry_f32.argtypes = [P, i64, i64, P]
        L.orc_y_entry_f32.restype = ctypes.c_double
        L.orc_compress_f64.argtypes = [u64, i64, i64, P, i64, i64, u64, P, P, i32]
        L.orc_compress_f32.argtypes = [u64, i64, i64, P, i64, i64, u64, P, P, i32]
        L.orc_gram_accumulate.argtypes = [i64, i64, P, P, i64, P, i32]
        L.orc_gram_rows.argtypes = [i64, i64, P, P, i64, P, i64, P, i32]
        L.orc_cov_finalize.argtypes = [i64, i64, i64, P, P]
        L.orc_kmeans_step.argtypes = [i64, i64, P, P, i64, i32, P, P, P, P, P, i32]
        L.orc_unmix.argtypes = [u64, i64, P, i32, P]
        L.orc_kmeanspp.argtypes = [u64, i64, i64, P, P, i64, i32, u64, P, P]
        L.orc_mean_estimate.argtypes = [i64, i64, P, P, i64, P]
        L.orc_kmeans_2pass.argtypes = [i64, P, i64, i32, P, P, P, P, P, i32]
        L.orc_max_threads.restype = i32
        L.orc_sample_batch.argtypes = [u64, u64, i64, i64, i64, P, i32]
        L.orc_sample_words_used.argtypes = [u64, u64, i64, i64]
        L.orc_gram_submatrix_f32.argtypes = [u64, i64, i64, P, i64, i64, u64, P, i64, P, i32]
        L.orc_sample_words_used.restype = i64
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(lib().orc_max_threads())


def philox4x64_10(counter, key):
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def lemire_from_words(rng: int, bits: int, words):
    w = np.ascontiguousarray(words, dtype=np.uint32)
    used = ctypes.c_int(0)
    r = lib().orc_lemire_from_words(rng, bits, _ptr(w), len(w), ctypes.byref(used))
    return int(r), int(used.value)


def floyd_from_draws(p: int, m: int, draws):
    d = np.ascontiguousarray(draws, dtype=np.uint32)
    idx = np.zeros(m, dtype=np.uint16)
    rc = lib().orc_floyd_from_draws(p, m, _ptr(d), _ptr(idx))
    if rc != 0:
        raise ValueError("invalid draw sequence")
    return idx


def sample_indices(seed: int, i: int, p: int, m: int):
    idx = np.zeros(m, dtype=np.uint16)
    lib().orc_sample_indices(seed, i, p, m, _ptr(idx))
    return idx


def sample_batch(seed: int, i0: int, n: int, p: int, m: int, nthreads: int = 0):
    idx = np.zeros((n, m), dtype=np.uint16)
    lib().orc_sample_batch(seed, i0, n, p, m, _ptr(idx), nthreads)
    return idx


def sample_words_used(seed: int, i: int, p: int, m: int) -> int:
    return int(lib().orc_sample_words_used(seed, i, p, m))


def signs(seed: int, p: int):
    D = np.zeros(p, dtype=np.int8)
    lib().orc_signs(seed, p, _ptr(D))
    return D


def fwht_normalized(v):
    a = np.array(v, dtype=np.float64, copy=True)
    lib().orc_fwht_normalized(_ptr(a), a.shape[-1])
    return a


def y_entry(seed: int, x, j: int, D=None):
    if D is None:
        D = signs(seed, x.shape[-1])
    D = np.ascontiguousarray(D, dtype=np.int8)
    if x.dtype == np.float32:
        xx = np.ascontiguousarray(x)
        return float(lib().orc_y_entry_f32(_ptr(D), xx.shape[-1], j, _ptr(xx)))
    xx = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().orc_y_entry_f64(_ptr(D), xx.shape[-1], j, _ptr(xx)))


def compress(X, seed: int, m: int, i0: int = 0, nthreads: int = 0):
    """Returns (vals float64 n x m, idx uint16 n x m)."""
    n, p = X.shape
    vals = np.zeros((n, m), dtype=np.float64)
    idx = np.zeros((n, m), dtype=np.uint16)
    if X.dtype == np.float32:
        Xc = np.ascontiguousarray(X)
        lib().orc_compress_f32(seed, p, m, _ptr(Xc), n, p, i0, _ptr(vals), _ptr(idx), nthreads)
    else:
        Xc = np.ascontiguousarray(X, dtype=np.float64)
        lib().orc_compress_f64(seed, p, m, _ptr(Xc), n, p, i0, _ptr(vals), _ptr(idx), nthreads)
    return vals, idx


def gram_accumulate(p: int, vals, idx, G=None, nthreads: int = 0):
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.uint16)
    n, m = vals.shape
    if G is None:
        G = np.zeros((p, p), dtype=np.float64)
    lib().orc_gram_accumulate(p, m, _ptr(vals), _ptr(idx), n, _ptr(G), nthreads)
    return G


def gram_rows(p: int, vals, idx, rows, nthreads: int = 0):
    """Rows `rows` of G = sum_i w_i w_i^T (len(rows) x p), each entry summed
    over the samples in order; the same sums as ``gram_accumulate``."""
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.uint16)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if len(np.unique(rows)) != len(rows) or (len(rows) and (rows.min() < 0 or rows.max() >= p)):
        raise ValueError("rows must be distinct coordinates in [0, p)")
    n, m = vals.shape
    out = np.zeros((len(rows), p), dtype=np.float64)
    lib().orc_gram_rows(p, m, _ptr(vals), _ptr(idx), n, _ptr(rows), len(rows), _ptr(out), nthreads)
    return out


def cov_rows(p: int, m: int, n: int, Grows, rows):
    """Rows `rows` of C_n from the matching rows of G (Sec. V): off-diagonal
    entries p(p-1)/(m(m-1)) G/n, the diagonal one p/(m n) G (the closed form of
    C_emp_hat - (p-m)/(p-1) diag(C_emp_hat))."""
    C = (p * (p - 1)) / (m * (m - 1)) * (np.asarray(Grows, dtype=np.float64) / n)
    r = np.arange(len(rows))
    C[r, rows] = C[r, rows] - (p - m) / (p - 1) * C[r, rows]
    return C


def gram_submatrix(seed: int, m: int, X, J, i0: int = 0, nthreads: int = 0):
    """G[J][J] from the definitions (explicit Hadamard rows, kept sets); X float32."""
    Xc = np.ascontiguousarray(X, dtype=np.float32)
    n, p = Xc.shape
    Jc = np.ascontiguousarray(J, dtype=np.int64)
    G = np.zeros((len(Jc), len(Jc)), dtype=np.float64)
    lib().orc_gram_submatrix_f32(seed, p, m, _ptr(Xc), n, p, i0, _ptr(Jc), len(Jc), _ptr(G), nthreads)
    return G


def cov_finalize(p: int, m: int, n: int, G):
    G = np.ascontiguousarray(G, dtype=np.float64)
    C = np.zeros((p, p), dtype=np.float64)
    lib().orc_cov_finalize(p, m, n, _ptr(G), _ptr(C))
    return C


def covariance(p: int, vals, idx, nthreads: int = 0):
    n, m = vals.shape
    return cov_finalize(p, m, n, gram_accumulate(p, vals, idx, nthreads=nthreads))


def kmeans_step(p: int, vals, idx, centers, nthreads: int = 0):
    """Returns (centers_out, assign int32, objective, margin)."""
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.uint16)
    cin = np.ascontiguousarray(centers, dtype=np.float64)
    n, m = vals.shape
    K = cin.shape[0]
    cout = np.zeros_like(cin)
    assign = np.zeros(n, dtype=np.int32)
    margin = np.zeros(n, dtype=np.float64)
    obj = ctypes.c_double(0.0)
    lib().orc_kmeans_step(p, m, _ptr(vals), _ptr(idx), n, K, _ptr(cin), _ptr(cout), _ptr(assign),
                          ctypes.byref(obj), _ptr(margin), nthreads)
    return cout, assign, float(obj.value), margin


def unmix(seed: int, centers_pre):
    c = np.ascontiguousarray(centers_pre, dtype=np.float64)
    K, p = c.shape
    out = np.zeros_like(c)
    lib().orc_unmix(seed, p, _ptr(c), K, _ptr(out))
    return out


def kmeanspp(seed: int, p: int, vals, idx, K: int, replicate: int = 0):
    """K-means++ seeding; starting point `replicate` draws its uniforms from
    the Philox blocks with counter (b, replicate, 2, 0)."""
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.uint16)
    n, m = vals.shape
    centers = np.zeros((K, p), dtype=np.float64)
    chosen = np.zeros(K, dtype=np.int64)
    lib().orc_kmeanspp(seed, p, m, _ptr(vals), _ptr(idx), n, K, replicate, _ptr(centers), _ptr(chosen))
    return centers, chosen


def kmeans_2pass(X, c_hat, mu_hat, nthreads: int = 0):
    """Returns (centers float64 K x p, assign int32 n, margin float64 n)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    c_hat = np.ascontiguousarray(c_hat, dtype=np.int32)
    mu_hat = np.ascontiguousarray(mu_hat, dtype=np.float64)
    n, p = X.shape
    K = mu_hat.shape[0]
    mu = np.zeros_like(mu_hat)
    c = np.zeros(n, dtype=np.int32)
    margin = np.zeros(n, dtype=np.float64)
    lib().orc_kmeans_2pass(p, _ptr(X), n, K, _ptr(c_hat), _ptr(mu_hat), _ptr(mu), _ptr(c), _ptr(margin), nthreads)
    return mu, c, margin


def mean_estimate(p: int, vals, idx):
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.uint16)
    n, m = vals.shape
    mean = np.zeros(p, dtype=np.float64)
    lib().orc_mean_estimate(p, m, _ptr(vals), _ptr(idx), n, _ptr(mean))
    return mean


def sparsified_kmeans_best(X, seed: int, m: int, K: int, T: int, R: int, nthreads: int = 0):
    """Alg. 1 with R random starting points on one compression: each start r
    is a K-means++ seeding (replicate r) followed by T rounds; the start whose
    last round reports the smallest objective (eq. CK_means; the earliest on
    ties) is kept.  Returns dict with best, objectives (R x T), centers_pre,
    assign, centers (unmixed) of the kept start."""
    n, p = X.shape
    vals, idx = compress(X, seed, m, nthreads=nthreads)
    out = kmeans_best_compressed(p, vals, idx, seed, K, T, R, nthreads)
    out.update({"vals": vals, "idx": idx, "centers": unmix(seed, out["centers_pre"])})
    return out


def kmeans_best_compressed(p: int, vals, idx, seed: int, K: int, T: int, R: int, nthreads: int = 0):
    """The R starts and the choice of ``sparsified_kmeans_best`` on given
    compressed samples (preconditioned domain)."""
    objs = np.zeros((R, T))
    best = None
    for r in range(R):
        mu, _ = kmeanspp(seed, p, vals, idx, K, r)
        assign = None
        for t in range(T):
            mu, assign, J, _ = kmeans_step(p, vals, idx, mu, nthreads=nthreads)
            objs[r, t] = J
        if best is None or objs[r, T - 1] < objs[best[0], T - 1]:
            best = (r, mu, assign)
    r, mu, assign = best
    return {"best": r, "objectives": objs, "centers_pre": mu, "assign": assign}


def dct_orthonormal(v):
    """y = C v with C the orthonormal DCT-II matrix (one of the fast
    orthonormal transforms Sec. III allows for H; the paper uses it for p = 784,
    Thm. 1 with eta = 1/2), along the last axis, by scipy's FFT-based DCT."""
    import scipy.fft

    return scipy.fft.dct(np.asarray(v, dtype=np.float64), type=2, norm="ortho", axis=-1)


def compress_dct(X, seed: int, m: int, i0: int = 0):
    """Alg. 1's first loop with the DCT in place of the Hadamard transform, for
    any p: y_i = C D x_i with the plan's signs D, then the kept sets of the
    sampler (the same (seed, i, p, m) streams).  Returns (vals n x m FP64,
    idx n x m uint16)."""
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    Y = dct_orthonormal(X * signs(seed, p).astype(np.float64))
    idx = sample_batch(seed, i0, n, p, m)
    return np.take_along_axis(Y, idx.astype(np.int64), axis=1), idx


def unmix_dct(seed: int, centers_pre):
    """mu = (C D)^T mu' = D C^T mu' for each row (the DCT form of eq. mu-mu')."""
    import scipy.fft

    c = np.asarray(centers_pre, dtype=np.float64)
    p = c.shape[-1]
    return scipy.fft.idct(c, type=2, norm="ortho", axis=-1) * signs(seed, p).astype(np.float64)


def clustering_accuracy(labels, assign, K: int):
    """Clustering accuracy of Sec. VII: the number of samples whose cluster
    matches their ground-truth label under the best one-to-one matching of
    clusters to labels, over n (the matching by the Hungarian method)."""
    from scipy.optimize import linear_sum_assignment

    labels = np.asarray(labels, dtype=np.int64)
    assign = np.asarray(assign, dtype=np.int64)
    M = np.zeros((K, K), dtype=np.int64)
    np.add.at(M, (assign, labels), 1)
    r, c = linear_sum_assignment(-M)
    return float(M[r, c].sum()) / len(labels)


def principal_components(C, k: int):
    """The k leading eigenvectors of the symmetric matrix C as the columns of a
    p x k matrix, eigenvalues descending (PCA on the estimate, Sec. V)."""
    w, V = np.linalg.eigh(np.asarray(C, dtype=np.float64))
    order = np.argsort(w)[::-1][:k]
    return np.ascontiguousarray(V[:, order])


def explained_variance(X, U):
    """Fraction of explained variance (Sec. II, comparison with column
    sampling): tr(U^T A A^T U) / tr(A A^T) for the p x n data matrix A whose
    columns are the samples and p x k orthonormal components U.  The samples
    are the rows of X here (A = X^T), so the fraction is ||X U||_F^2 / ||X||_F^2."""
    X = np.asarray(X, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    P = X @ U
    return float(np.sum(P * P) / np.sum(X * X))


def sparsified_kmeans(X, seed: int, m: int, K: int, T: int, init_centers=None, nthreads: int = 0):
    """Alg. 1: compress once, seed, T assignment/update rounds, unmix.

    Returns dict with vals, idx, centers_pre (per step list), assign, objectives,
    centers (unmixed).
    """
    n, p = X.shape
    vals, idx = compress(X, seed, m, nthreads=nthreads)
    if init_centers is None:
        init_centers, _ = kmeanspp(seed, p, vals, idx, K)
    mu = init_centers
    objs = []
    assign = None
    for _ in range(T):
        mu, assign, J, _ = kmeans_step(p, vals, idx, mu, nthreads=nthreads)
        objs.append(J)
    return {"vals": vals, "idx": idx, "centers_pre": mu, "assign": assign,
            "objectives": objs, "centers": unmix(seed, mu), "init": init_centers}
