"""Preconditioned data sparsification on MI355X (gfx950).

Python face of libpds (C ABI in include/pds.h).  Tensors are torch tensors on
the current HIP device; every call enqueues the library's kernels on
``torch.cuda.current_stream()`` and returns without synchronising.

    plan = Plan(p, m, seed, PDS_F32)
    vals, idx = compress(plan, X)              # Alg. 1 first loop (Sec. III, eq. ROS)
    C = covariance(plan, vals, idx)            # Sec. V, unbiased C_n (preconditioned domain)
    mu, c, J = kmeans_step(plan, vals, idx, mu0)   # Sec. VI, one Lloyd round
    centers = unmix(plan, mu)                  # eq. mu-mu'
    mu0, chosen = kmeanspp(plan, vals, idx, K) # Alg. 1 seeding (K-means++)
    xbar = sample_mean(plan, vals, idx)        # Sec. IV (preconditioned domain)
"""
import ctypes

from ._lib import (PDS_E_ARG, PDS_E_HIP, PDS_E_M, PDS_E_UNSUPPORTED, PDS_E_WORKSPACE, PDS_EXPLAINED_WS_BYTES, PDS_F32,
                   PDS_F64, PDS_GRAM_AUTO, PDS_GRAM_DENSE, PDS_GRAM_SPARSE, PDS_OK, PDS_OP_COMPRESS, PDS_OP_COVARIANCE, PDS_OP_KMEANS, PDS_OP_KMEANS2, PDS_OP_KMEANS_BEST, PDS_OP_KMEANS_RUN,
                   PDS_OP_KMEANSPP, PDS_OP_MEAN, PDS_SPLIT_BF16, PDS_TRANSFORM_DCT, PDS_TRANSFORM_HADAMARD, PDS_DCT_MAX_P,
                   EXPORTS, PdsError, check, lib)

__all__ = [
    "Plan", "compress", "pad_rows", "covariance", "CovarianceAccumulator", "sample_mean", "kmeanspp", "kmeans_best",
    "kmeans_step", "kmeans_run", "unmix", "kmeans_2pass", "sparsified_kmeans", "top_eigenvalues", "principal_components",
    "explained_variance",
    "PdsError", "PDS_F64", "PDS_F32", "PDS_SPLIT_BF16", "PDS_GRAM_AUTO", "PDS_GRAM_DENSE", "PDS_GRAM_SPARSE", "lib",
    "PDS_TRANSFORM_HADAMARD", "PDS_TRANSFORM_DCT", "PDS_DCT_MAX_P", "EXPORTS",
]


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """pds_plan: dimension p, kept coordinates m, seed, precision, the
    covariance's Gram form (PDS_GRAM_AUTO, PDS_GRAM_DENSE or PDS_GRAM_SPARSE)
    and the preconditioner (PDS_TRANSFORM_HADAMARD, p a power of two, or
    PDS_TRANSFORM_DCT, any p up to PDS_DCT_MAX_P)."""

    def __init__(self, p: int, m: int, seed: int = 0, prec: int = PDS_F32, gram: int = PDS_GRAM_AUTO,
                 transform: int = PDS_TRANSFORM_HADAMARD):
        self.p, self.m, self.seed, self.prec = int(p), int(m), int(seed), int(prec)
        self.transform = int(transform)
        h = ctypes.c_void_p()
        if self.transform == PDS_TRANSFORM_DCT:
            check(lib().pds_plan_create_dct(ctypes.byref(h), self.p, self.m, self.seed, self.prec),
                  "pds_plan_create_dct")
        else:
            check(lib().pds_plan_create(ctypes.byref(h), self.p, self.m, self.seed, self.prec), "pds_plan_create")
        self._h = h
        if gram != PDS_GRAM_AUTO:
            check(lib().pds_plan_set_gram(h, int(gram)), "pds_plan_set_gram")
        b = ctypes.c_size_t(0)
        check(lib().pds_covariance_acc_size(h, ctypes.byref(b)), "pds_covariance_acc_size")
        self.pg = int(round((b.value // 8) ** 0.5))  # the covariance accumulator is pg x pg

    def gram_form(self, n: int) -> int:
        """PDS_GRAM_DENSE or PDS_GRAM_SPARSE: the form a covariance call over n samples runs."""
        a = ctypes.c_int32(0)
        check(lib().pds_plan_gram(self._h, int(n), ctypes.byref(a)), "pds_plan_gram")
        return int(a.value)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().pds_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dtype(self):
        import torch

        return torch.float64 if self.prec == PDS_F64 else torch.float32

    def signs(self):
        import numpy as np

        D = np.zeros(self.p, dtype=np.int8)
        check(lib().pds_signs(self._h, D.ctypes.data_as(ctypes.c_void_p)), "pds_signs")
        return D

    def workspace_size(self, op: int, n: int, K: int = 1) -> int:
        b = ctypes.c_size_t(0)
        check(lib().pds_workspace_size(self._h, int(op), int(n), int(K), ctypes.byref(b)), "pds_workspace_size")
        return int(b.value)

    def workspace(self, op: int, n: int, K: int = 1, device=None):
        import torch

        nb = self.workspace_size(op, n, K)
        if nb == 0:
            return None
        return torch.empty(nb, dtype=torch.uint8, device=device or "cuda")


def pad_rows(X, p_pad: int, out=None):
    """Rows of X (n x p_data, p_data <= p_pad) zero-padded to width p_pad on
    the device (pds_pad_rows)."""
    import torch

    n, pd = X.shape
    if X.stride(1) != 1:
        raise ValueError("X rows must be contiguous")
    if out is None:
        out = torch.empty((n, int(p_pad)), dtype=X.dtype, device=X.device)
    xp = PDS_F64 if X.dtype == torch.float64 else PDS_F32
    check(lib().pds_pad_rows(_ptr(X), xp, n, pd, X.stride(0), _ptr(out), int(p_pad), _stream()), "pds_pad_rows")
    return out


def compress(plan: Plan, X, i0: int = 0, vals=None, idx=None, ws=None):
    """Returns (vals n x m, idx n x m uint16 as torch.int16 storage).  For a
    Hadamard plan, rows narrower than the plan's p (a dimension that is not a
    power of two) are zero-padded first (pad_rows); a DCT plan takes rows of
    exactly its p."""
    import torch

    n, p = X.shape
    if p < plan.p and plan.transform == PDS_TRANSFORM_HADAMARD:
        X = pad_rows(X, plan.p)
        p = plan.p
    if p != plan.p:
        raise ValueError(f"X has {p} columns, plan has p={plan.p}")
    if X.dtype != plan.dtype:
        raise TypeError(f"X dtype {X.dtype} does not match plan dtype {plan.dtype}")
    if X.stride(1) != 1:
        raise ValueError("X rows must be contiguous")
    if vals is None:
        vals = torch.empty((n, plan.m), dtype=plan.dtype, device=X.device)
    if idx is None:
        idx = torch.empty((n, plan.m), dtype=torch.int16, device=X.device)
    if ws is None:
        ws = plan.workspace(PDS_OP_COMPRESS, n, device=X.device)
    wsb = ws.numel() if ws is not None else 0
    check(lib().pds_compress(plan.handle, _ptr(X), n, X.stride(0), int(i0), _ptr(vals), _ptr(idx), _ptr(ws), wsb,
                             _stream()), "pds_compress")
    return vals, idx


class CovarianceAccumulator:
    """Streaming covariance (Sec. V): add batches, then finalize."""

    def __init__(self, plan: Plan, device=None):
        import torch

        self.plan = plan
        self.acc = torch.zeros((plan.pg, plan.pg), dtype=torch.float64, device=device or "cuda")
        self.n = 0
        self._ws = None

    def _workspace(self, n, device):
        need = self.plan.workspace_size(PDS_OP_COVARIANCE, n)
        if need and (self._ws is None or self._ws.numel() < need):
            import torch

            self._ws = torch.empty(need, dtype=torch.uint8, device=device)
        return self._ws

    def add(self, vals, idx):
        n = vals.shape[0]
        ws = self._workspace(n, vals.device)
        check(lib().pds_covariance(self.plan.handle, _ptr(vals), _ptr(idx), n, _ptr(self.acc), 0, 0,
                                   ctypes.c_void_p(0), _ptr(ws), ws.numel() if ws is not None else 0, _stream()),
              "pds_covariance")
        self.n += n
        return self

    def finalize(self, C=None):
        import torch

        if C is None:
            C = torch.empty((self.plan.p, self.plan.p), dtype=torch.float64, device=self.acc.device)
        check(lib().pds_covariance(self.plan.handle, ctypes.c_void_p(0), ctypes.c_void_p(0), 0, _ptr(self.acc), 1,
                                   self.n, _ptr(C), ctypes.c_void_p(0), 0, _stream()), "pds_covariance")
        return C


def covariance(plan: Plan, vals, idx, acc=None, ws=None, C=None):
    """Unbiased covariance estimate C_n (p x p FP64) of the compressed samples."""
    import torch

    n = vals.shape[0]
    dev = vals.device
    if acc is None:
        acc = torch.zeros((plan.pg, plan.pg), dtype=torch.float64, device=dev)
    if C is None:
        C = torch.empty((plan.p, plan.p), dtype=torch.float64, device=dev)
    if acc.dtype != torch.float64 or acc.numel() < plan.pg * plan.pg or not acc.is_contiguous():
        raise ValueError(f"acc must be a contiguous FP64 buffer of {plan.pg} x {plan.pg}")
    if C.dtype != torch.float64 or C.numel() < plan.p * plan.p or not C.is_contiguous():
        raise ValueError(f"C must be a contiguous FP64 buffer of {plan.p} x {plan.p}")
    if ws is None:
        ws = plan.workspace(PDS_OP_COVARIANCE, n, device=dev)
    check(lib().pds_covariance(plan.handle, _ptr(vals), _ptr(idx), n, _ptr(acc), 1, n, _ptr(C), _ptr(ws),
                               ws.numel() if ws is not None else 0, _stream()), "pds_covariance")
    return C


def sample_mean(plan: Plan, vals, idx, acc=None, finalize: bool = True, n_total=None, out=None, ws=None):
    """Sample-mean estimate (Sec. IV) of the compressed samples, in the
    preconditioned domain: acc (p FP64, zeroed when None) += the per-coordinate
    sums of vals; when finalize, returns (p/(m n_total)) acc (n_total defaults
    to this batch's n), else returns acc."""
    import torch

    n = vals.shape[0]
    dev = vals.device
    if acc is None:
        acc = torch.zeros(plan.p, dtype=torch.float64, device=dev)
    if n_total is None:
        n_total = n
    if finalize and out is None:
        out = torch.empty(plan.p, dtype=torch.float64, device=dev)
    if ws is None:
        ws = plan.workspace(PDS_OP_MEAN, n, device=dev)
    check(lib().pds_sample_mean(plan.handle, _ptr(vals), _ptr(idx), n, _ptr(acc), 1 if finalize else 0, n_total,
                                _ptr(out), _ptr(ws), ws.numel() if ws is not None else 0,
                                _stream()), "pds_sample_mean")
    return out if finalize else acc


def top_eigenvalues(C, k: int = 20):
    """The k largest eigenvalues (descending, FP64) of the symmetric, possibly
    indefinite covariance estimate C (PCA on the estimate, Sec. V): the
    device's dense symmetric eigensolver (rocSOLVER through torch.linalg) on
    the FP64 matrix where it lives.  Eigenvalues are the same in the
    preconditioned and the original domain (H D is orthogonal)."""
    import torch

    if C.dim() != 2 or C.shape[0] != C.shape[1]:
        raise ValueError("C must be square")
    w = torch.linalg.eigvalsh(C.to(torch.float64))
    k = min(int(k), C.shape[0])
    return torch.flip(w, dims=[0])[:k]


def principal_components(plan: Plan, C, k: int):
    """PCA on the covariance estimate (Sec. V): the k leading eigenvectors of
    C (p x p FP64, preconditioned domain) from the device's symmetric
    eigensolver (rocSOLVER through torch.linalg), mapped back to the original
    domain by pds_unmix.  Returns (components k x p FP64, rows orthonormal;
    eigenvalues (k,) descending)."""
    import torch

    k = int(k)
    if C.dim() != 2 or C.shape[0] != C.shape[1] or C.shape[0] != plan.p or not 1 <= k <= plan.p:
        raise ValueError("C must be p x p and 1 <= k <= p")
    w, V = torch.linalg.eigh(C.to(torch.float64))
    top = torch.flip(V[:, -k:], dims=[1]).T.contiguous()
    return unmix(plan, top), torch.flip(w[-k:], dims=[0])


def explained_variance(X, comps, out=None, ws=None):
    """Fraction of explained variance (Sec. II) of the components `comps`
    (k x p FP64, orthonormal rows) over the rows of X (n x p, FP32 or FP64):
    returns the device tensor (||X comps^T||_F^2, ||X||_F^2) (2,) FP64."""
    import torch

    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D tensor with unit column stride")
    if X.dtype not in (torch.float32, torch.float64) or comps.dtype != torch.float64:
        raise TypeError("X must be FP32 or FP64 and comps FP64")
    comps = comps.contiguous()
    if ws is None:
        ws = torch.empty(PDS_EXPLAINED_WS_BYTES, dtype=torch.uint8, device=X.device)
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=X.device)
    xp = PDS_F64 if X.dtype == torch.float64 else PDS_F32
    check(lib().pds_explained_variance(_ptr(comps), comps.shape[0], _ptr(X), xp, X.shape[0], X.shape[1], X.stride(0),
                                       _ptr(out), _ptr(ws), ws.numel(), _stream()), "pds_explained_variance")
    return out


def kmeanspp(plan: Plan, vals, idx, K: int, centers=None, chosen=None, ws=None, replicate: int = 0):
    """K-means++ seeding (Alg. 1) on the compressed samples with the plan's
    seed and starting point `replicate`: returns (centers K x p FP64,
    zero-filled compressed vectors of the chosen samples; chosen (K,) int64)."""
    import torch

    n = vals.shape[0]
    dev = vals.device
    K = int(K)
    if centers is None:
        centers = torch.empty((K, plan.p), dtype=torch.float64, device=dev)
    if chosen is None:
        chosen = torch.empty(K, dtype=torch.int64, device=dev)
    if ws is None:
        ws = plan.workspace(PDS_OP_KMEANSPP, n, device=dev)
    check(lib().pds_kmeanspp(plan.handle, _ptr(vals), _ptr(idx), n, K, int(replicate), _ptr(centers), _ptr(chosen),
                             _ptr(ws), ws.numel() if ws is not None else 0, _stream()), "pds_kmeanspp")
    return centers, chosen


def kmeans_best(plan: Plan, vals, idx, K: int, T: int, R: int, ws=None):
    """Sparsified K-means from R K-means++ starting points, T rounds each, the
    start with the smallest final objective kept (all on the device): returns
    (centers K x p FP64 preconditioned domain, assign (n,) int32, objectives
    (R, T) FP64, best (1,) int32)."""
    import torch

    n = vals.shape[0]
    dev = vals.device
    centers = torch.empty((int(K), plan.p), dtype=torch.float64, device=dev)
    assign = torch.empty(n, dtype=torch.int32, device=dev)
    objs = torch.empty((int(R), int(T)), dtype=torch.float64, device=dev)
    best = torch.empty(1, dtype=torch.int32, device=dev)
    if ws is None:
        ws = plan.workspace(PDS_OP_KMEANS_BEST, n, int(K), device=dev)
    check(lib().pds_kmeans_best(plan.handle, _ptr(vals), _ptr(idx), n, int(K), int(T), int(R), _ptr(centers),
                                _ptr(assign), _ptr(objs), _ptr(best), _ptr(ws), ws.numel() if ws is not None else 0,
                                _stream()), "pds_kmeans_best")
    return centers, assign, objs, best


def kmeans_step(plan: Plan, vals, idx, centers, out=None, assign=None, objective=None, ws=None):
    """One sparsified Lloyd round; returns (centers_out, assign int32, objective (1,) FP64)."""
    import torch

    n = vals.shape[0]
    K = centers.shape[0]
    dev = vals.device
    if out is None:
        out = torch.empty_like(centers)
    if assign is None:
        assign = torch.empty(n, dtype=torch.int32, device=dev)
    if objective is None:
        objective = torch.empty(1, dtype=torch.float64, device=dev)
    if ws is None:
        ws = plan.workspace(PDS_OP_KMEANS, n, K, device=dev)
    check(lib().pds_kmeans_step(plan.handle, _ptr(vals), _ptr(idx), n, K, _ptr(centers), _ptr(out), _ptr(assign),
                                _ptr(objective), _ptr(ws), ws.numel() if ws is not None else 0, _stream()),
          "pds_kmeans_step")
    return out, assign, objective


def kmeans_run(plan: Plan, vals, idx, centers, T: int, out=None, assign=None, objectives=None, ws=None):
    """T sparsified Lloyd rounds from `centers` (Alg. 1's loop, pds_kmeans_run);
    returns (centers after the last round, its assign int32, objectives (T,)
    FP64, round t's with the centers entering it)."""
    import torch

    n = vals.shape[0]
    K = centers.shape[0]
    dev = vals.device
    if out is None:
        out = torch.empty_like(centers)
    if assign is None:
        assign = torch.empty(n, dtype=torch.int32, device=dev)
    if objectives is None:
        objectives = torch.empty(int(T), dtype=torch.float64, device=dev)
    if ws is None:
        ws = plan.workspace(PDS_OP_KMEANS_RUN, n, K, device=dev)
    check(lib().pds_kmeans_run(plan.handle, _ptr(vals), _ptr(idx), n, K, int(T), _ptr(centers), _ptr(out),
                               _ptr(assign), _ptr(objectives), _ptr(ws), ws.numel() if ws is not None else 0,
                               _stream()), "pds_kmeans_run")
    return out, assign, objectives


def unmix(plan: Plan, centers_pre, out=None):
    """mu = (H D)^T mu' (DCT plans: (C D)^T mu') for each row of centers_pre (FP64)."""
    import torch

    if out is None:
        out = torch.empty_like(centers_pre)
    check(lib().pds_unmix(plan.handle, _ptr(centers_pre), centers_pre.shape[0], _ptr(out), _stream()), "pds_unmix")
    return out


def kmeans_2pass(plan: Plan, X, c_hat, mu_hat, out=None, assign=None, ws=None):
    """Second pass of two-pass sparsified K-means over the original rows X
    (n x p; FP64 for FP64 plans, FP32 otherwise): returns (centers K x p FP64,
    the means of the rows of each one-pass cluster c_hat; assign int32, the
    nearest one-pass center mu_hat in the original domain)."""
    import torch

    n, p = X.shape
    K = mu_hat.shape[0]
    dev = X.device
    if out is None:
        out = torch.empty_like(mu_hat)
    if assign is None:
        assign = torch.empty(n, dtype=torch.int32, device=dev)
    if ws is None:
        ws = plan.workspace(PDS_OP_KMEANS2, n, K, device=dev)
    check(lib().pds_kmeans_2pass(plan.handle, _ptr(X), n, X.stride(0), K, _ptr(c_hat), _ptr(mu_hat), _ptr(out),
                                 _ptr(assign), _ptr(ws), ws.numel() if ws is not None else 0, _stream()),
          "pds_kmeans_2pass")
    return out, assign


def sparsified_kmeans(plan: Plan, X, init_centers, iterations: int, starts: int = 1):
    """Alg. 1: one compression pass, `iterations` assignment/update rounds,
    unmixing.  init_centers: K x p FP64 initial centers (preconditioned
    domain), or an int K to seed on the device with K-means++ (with
    starts > 1, the best of that many K-means++ starts is kept; objectives is
    then starts x iterations).  Returns dict(vals, idx, assign, centers_pre,
    centers, objectives)."""
    import torch

    vals, idx = compress(plan, X)
    if isinstance(init_centers, int):
        K = init_centers
        if starts > 1:
            c, assign, objs, best = kmeans_best(plan, vals, idx, K, iterations, starts)
            return {"vals": vals, "idx": idx, "assign": assign, "centers_pre": c, "centers": unmix(plan, c),
                    "objectives": objs, "best": best}
        init_centers, _ = kmeanspp(plan, vals, idx, K)
    a, assign, objs = kmeans_run(plan, vals, idx, init_centers, iterations)
    return {"vals": vals, "idx": idx, "assign": assign, "centers_pre": a, "centers": unmix(plan, a),
            "objectives": objs}
