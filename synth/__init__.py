"""Seeded synthetic inputs for the workloads (shared by tests and the bench).

This module holds no step of the method: it only draws data matrices X (one
sample per row, row-major n x p) and model parameters.  Both the GPU path and
the CPU oracle receive the same bytes from here.

Workloads (shapes and distributions follow the paper's synthetic generators;
the paper's public datasets are not used):

* ``spiked`` -- x_i = U diag(sqrt(lam)) kappa_i + eps_i, U the Q factor of a
  p x k standard-normal matrix, kappa, eps ~ N(0, 1): the principal-component
  generator of Sec. V (numerical experiment of Thm. "covariance").
  Small case: p = 256, k = 5, lam = (50, 40, 30, 20, 10), n = 2000, FP64.
  Precision case: p = 4096, k = 20, lam_k = 50 / k, n = 2^20, FP32.
* ``mixture`` -- K Gaussian clusters, centers N(0, 4 I), unit within-cluster
  variance, each entry replaced with probability 1% by 20 * t_3 (heavy-tailed
  spikes, the "few large entries" case that motivates preconditioning):
  p = 1024, K = 10, n = 2^20, FP32.

* ``batch256_f32`` -- the batched form's 256 independent sets: n ~ U{1000..100000},
  p ~ U{128, 256, 512, 1024, 2048}, K ~ U{2..50}, gamma ~ U[0.02, 0.2], each set
  drawn like ``mixture`` with its own K centers; 20 K-means rounds.
* ``digits784_f32`` -- stand-in for the handwritten-digit images of Sec. VII
  (70000 images of 28 x 28 = 784 pixels, 10 classes; the dataset itself is
  not used): each class is a template of five Gaussian blobs (width 1.3
  pixels) placed in the central 20 x 20 pixels; a sample shifts its class
  template by up to 2 pixels each way, scales it by U[0.7, 1.3], adds
  N(0, 0.1^2) noise, clips to [0, 1] and zeroes pixels below 0.15 (about a
  fifth of the pixels stay non-zero, as in the images).  p = 784 is not a
  power of two: the paper preconditions such data with a DCT.
* ``msel`` -- data blocks for the learned m-selector (not a workload of the
  paper): p = 1024, n = 8192, spike rank r ~ U{1..50}, lam_k = A / k with
  amplitude A log-uniform on [50, 5e4], unit noise.  The principal directions
  mix a random orthonormal basis with r canonical basis vectors, weight alpha ~
  U[0, 1] on the canonical part, re-orthonormalized: alpha = 1 gives maximally
  coherent data (the canonical-PC case of Sec. V's Table 1), alpha = 0
  incoherent data.

Row blocks are drawn from per-block generators (block = 65536 rows) so any
leading slice of a workload is identical to the same rows of the full one.
"""
import math

import numpy as np

BLOCK = 65536

WORKLOADS = {
    # name: dict of shape/distribution parameters
    "small_f64": dict(kind="spiked", n=2000, p=256, lam=(50.0, 40.0, 30.0, 20.0, 10.0),
                      dtype="f64", data_seed=0, gamma=0.1, K=5, T=10),
    "mixture_f32": dict(kind="mixture", n=1 << 20, p=1024, K=10, center_std=2.0, spike_prob=0.01,
                        spike_scale=20.0, spike_dof=3, dtype="f32", data_seed=1, gamma=0.05, T=20),
    "spiked4096_f32": dict(kind="spiked", n=1 << 20, p=4096, lam=tuple(50.0 / k for k in range(1, 21)),
                           dtype="f32", data_seed=2, gamma=0.1),
    "digits784_f32": dict(kind="digits", n=70000, p=784, K=10, side=28, strokes=5, width=1.3, shift=2,
                          noise=0.1, floor=0.15, dtype="f32", data_seed=4, gamma=0.1, T=20),
    "batch256_f32": dict(kind="batch", count=256, n=(1000, 100000), p=(128, 256, 512, 1024, 2048), K=(2, 50),
                         gamma=(0.02, 0.2), center_std=2.0, spike_prob=0.01, spike_scale=20.0, spike_dof=3,
                         dtype="f32", data_seed=3, T=20),
}


def digits_numpy(name="digits784_f32", n=None, with_labels=False):
    """Rows of the digit-image stand-in (see the module notes), float32 in
    [0, 1], drawn with numpy from the workload's data seed."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    side, K = w["side"], w["K"]
    rng = np.random.default_rng([w["data_seed"], 0xD161])
    yy, xx = np.mgrid[0:side, 0:side].astype(np.float64)
    templ = np.zeros((K, side, side))
    for k in range(K):
        for _ in range(w["strokes"]):
            cy, cx = rng.uniform(4, side - 4, size=2)
            templ[k] += np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * w["width"] ** 2))
        templ[k] /= templ[k].max()
    labels = rng.integers(0, K, size=n)
    sh = rng.integers(-w["shift"], w["shift"] + 1, size=(n, 2))
    amp = rng.uniform(0.7, 1.3, size=n)
    X = np.empty((n, side * side), dtype=np.float32)
    for r0 in range(0, n, 8192):
        r1 = min(n, r0 + 8192)
        img = np.empty((r1 - r0, side, side))
        for i in range(r0, r1):
            img[i - r0] = np.roll(templ[labels[i]], (sh[i, 0], sh[i, 1]), axis=(0, 1)) * amp[i]
        img += w["noise"] * rng.standard_normal(img.shape)
        img = np.clip(img, 0.0, 1.0)
        img[img < w["floor"]] = 0.0
        X[r0:r1] = img.reshape(r1 - r0, -1)
    if with_labels:
        return X, labels
    return X


def m_from_gamma(gamma, p):
    """m = floor(gamma * p + 1/2): m must be a natural number (Cor. sampleMean)."""
    return int(math.floor(gamma * p + 0.5))


def model(name):
    """Model parameters (numpy float64), from the workload's data seed."""
    w = WORKLOADS[name]
    rng = np.random.default_rng([w["data_seed"], 0xA11CE])
    p = w["p"]
    if w["kind"] == "spiked":
        k = len(w["lam"])
        U, _ = np.linalg.qr(rng.standard_normal((p, k)))
        return {"U": U, "lam": np.asarray(w["lam"], dtype=np.float64)}
    centers = w["center_std"] * rng.standard_normal((w["K"], p))
    return {"centers": centers}


def _block_numpy(name, b, rows, mdl):
    w = WORKLOADS[name]
    p = w["p"]
    rng = np.random.default_rng([w["data_seed"], 0xB10C, b])
    if w["kind"] == "spiked":
        U, lam = mdl["U"], mdl["lam"]
        kappa = rng.standard_normal((rows, len(lam)))
        X = (kappa * np.sqrt(lam)) @ U.T + rng.standard_normal((rows, p))
        labels = None
    else:
        labels = rng.integers(0, w["K"], size=rows)
        X = mdl["centers"][labels] + rng.standard_normal((rows, p))
        mask = rng.random((rows, p)) < w["spike_prob"]
        nspk = int(mask.sum())
        X[mask] = w["spike_scale"] * rng.standard_t(w["spike_dof"], size=nspk)
    return X, labels


def rows_numpy(name, n=None, mdl=None, with_labels=False):
    """First n rows of the workload as a numpy array of the workload dtype."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    mdl = model(name) if mdl is None else mdl
    dt = np.float64 if w["dtype"] == "f64" else np.float32
    X = np.empty((n, w["p"]), dtype=dt)
    labels = np.empty(n, dtype=np.int64) if w["kind"] == "mixture" else None
    for b in range((n + BLOCK - 1) // BLOCK):
        r0 = b * BLOCK
        r1 = min(n, r0 + BLOCK)
        Xb, lb = _block_numpy(name, b, BLOCK, mdl)
        X[r0:r1] = Xb[: r1 - r0]
        if labels is not None:
            labels[r0:r1] = lb[: r1 - r0]
    if with_labels:
        return X, labels
    return X


def rows_torch(name, n=None, device="cuda", seed_offset=0):
    """The workload drawn with torch on `device` (fast for the full sizes).

    Same distribution and model parameters as rows_numpy, different random
    stream (torch's generator), so the bytes differ from rows_numpy's.
    """
    import torch

    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    p = w["p"]
    mdl = model(name)
    dt = torch.float64 if w["dtype"] == "f64" else torch.float32
    g = torch.Generator(device=device)
    g.manual_seed(w["data_seed"] * 1000003 + 17 + seed_offset)
    X = torch.empty((n, p), dtype=dt, device=device)
    step = BLOCK
    if w["kind"] == "spiked":
        U = torch.as_tensor(mdl["U"], dtype=torch.float32, device=device)
        sl = torch.as_tensor(np.sqrt(mdl["lam"]), dtype=torch.float32, device=device)
        for r0 in range(0, n, step):
            r1 = min(n, r0 + step)
            kappa = torch.randn((r1 - r0, len(sl)), generator=g, device=device)
            blk = (kappa * sl) @ U.T
            blk += torch.randn((r1 - r0, p), generator=g, device=device)
            X[r0:r1] = blk.to(dt)
    else:
        C = torch.as_tensor(mdl["centers"], dtype=torch.float32, device=device)
        for r0 in range(0, n, step):
            r1 = min(n, r0 + step)
            rows = r1 - r0
            lab = torch.randint(0, w["K"], (rows,), generator=g, device=device)
            blk = C[lab] + torch.randn((rows, p), generator=g, device=device)
            mask = torch.rand((rows, p), generator=g, device=device) < w["spike_prob"]
            # Student t with nu dof: Z / sqrt(chi2_nu / nu), chi2 from nu squared normals
            z = torch.randn((rows, p), generator=g, device=device)
            chi = torch.zeros((rows, p), device=device)
            for _ in range(w["spike_dof"]):
                chi += torch.randn((rows, p), generator=g, device=device) ** 2
            t = z / torch.sqrt(chi / w["spike_dof"])
            blk = torch.where(mask, w["spike_scale"] * t, blk)
            X[r0:r1] = blk.to(dt)
    return X


def random_compressed(n, p, m, seed, dtype=np.float32, K=None):
    """Synthetic compressed data for step-level tests: sorted distinct indices
    per row (numpy's own sampler) and normal values, plus optional K centers.
    The values are representable in `dtype` (so both sides can read the same
    numbers)."""
    rng = np.random.default_rng([seed, 0xC0DE])
    idx = np.empty((n, m), dtype=np.uint16)
    for i in range(n):
        idx[i] = np.sort(rng.choice(p, size=m, replace=False))
    vals = rng.standard_normal((n, m)).astype(dtype)
    out = {"vals": vals, "idx": idx}
    if K is not None:
        out["centers"] = rng.standard_normal((K, p)) * 0.5
    return out


# ---------------------------------------------------------------------------
# m-selector blocks
# ---------------------------------------------------------------------------
MSEL = dict(p=1024, n=8192, rank=(1, 50), amp=(50.0, 5.0e4), target=0.1, nsub=512, gamma_baseline=0.2,
            data_seed=5)


def msel_block_params(seed, b):
    """Parameters of block b of stream `seed`: rank r, coherence weight alpha, amplitude A."""
    rng = np.random.default_rng([MSEL["data_seed"], seed, b, 0xE3])
    lo, hi = MSEL["rank"]
    r = int(rng.integers(lo, hi + 1))
    alpha = float(rng.uniform())
    a0, a1 = MSEL["amp"]
    A = float(math.exp(rng.uniform(math.log(a0), math.log(a1))))
    return {"r": r, "alpha": alpha, "amp": A}


def msel_basis(seed, b, p, prm):
    """p x r orthonormal principal directions of block b: the Q factor of
    (1 - alpha) G / sqrt(p) + alpha E, G standard normal, E r distinct
    canonical basis vectors (Gaussian columns over sqrt(p) are already close
    to orthonormal; the QR makes them exactly so)."""
    rng = np.random.default_rng([MSEL["data_seed"], seed, b, 0xBA5E])
    r, alpha = prm["r"], prm["alpha"]
    E = np.zeros((p, r))
    E[rng.choice(p, size=r, replace=False), np.arange(r)] = 1.0
    A = (1.0 - alpha) * rng.standard_normal((p, r)) / math.sqrt(p) + alpha * E
    U, _ = np.linalg.qr(A)
    return U


def msel_block_numpy(seed, b, p=None, n=None):
    """Block b of stream `seed` as float32 numpy (n x p), and its parameters."""
    p = MSEL["p"] if p is None else p
    n = MSEL["n"] if n is None else n
    prm = msel_block_params(seed, b)
    prm["r"] = min(prm["r"], p)
    U = msel_basis(seed, b, p, prm)
    lam = prm["amp"] / np.arange(1, prm["r"] + 1)
    rng = np.random.default_rng([MSEL["data_seed"], seed, b, 0xDA7A])
    X = (rng.standard_normal((n, prm["r"])) * np.sqrt(lam)) @ U.T + rng.standard_normal((n, p))
    return X.astype(np.float32), prm


def msel_blocks_torch(seed, b0, count, p=None, n=None, device="cuda"):
    """Blocks b0 .. b0+count-1 drawn with torch on `device` (same parameters
    and construction as msel_block_numpy, torch's generator for every draw).
    The bases come from one batched QR of 50-column matrices: the first r
    columns of a Q factor depend only on the first r columns of its input, so
    block b keeps the first r columns.  Yields (X, params) per block."""
    import torch

    p = MSEL["p"] if p is None else p
    n = MSEL["n"] if n is None else n
    R = min(MSEL["rank"][1], p)
    prms = [msel_block_params(seed, b) for b in range(b0, b0 + count)]
    g = torch.Generator(device=device)
    g.manual_seed((MSEL["data_seed"] * 1000003 + seed) * 1000003 + b0)
    alpha = torch.tensor([q["alpha"] for q in prms], dtype=torch.float32, device=device).view(-1, 1, 1)
    rows = torch.rand((count, p), generator=g, device=device).argsort(dim=1)[:, :R]
    E = torch.zeros((count, p, R), device=device)
    E.scatter_(1, rows.unsqueeze(1), 1.0)
    A = (1.0 - alpha) * torch.randn((count, p, R), generator=g, device=device) / math.sqrt(p) + alpha * E
    Q, _ = torch.linalg.qr(A)
    for k, prm in enumerate(prms):
        prm["r"] = min(prm["r"], p)
        r = prm["r"]
        sl = torch.as_tensor(np.sqrt(prm["amp"] / np.arange(1, r + 1)), dtype=torch.float32, device=device)
        Z = torch.randn((n, r), generator=g, device=device)
        X = torch.randn((n, p), generator=g, device=device)
        X.addmm_(Z * sl, Q[k, :, :r].T)
        yield X, prm


# ---------------------------------------------------------------------------
# batched sets
# ---------------------------------------------------------------------------
def batch_params(name="batch256_f32", count=None):
    """Per-set (n, p, K, gamma, m) of a batched workload, from its data seed."""
    w = WORKLOADS[name]
    rng = np.random.default_rng([w["data_seed"], 0xBA7C])
    out = []
    for i in range(w["count"] if count is None else count):
        n = int(rng.integers(w["n"][0], w["n"][1] + 1))
        p = int(rng.choice(w["p"]))
        K = int(rng.integers(w["K"][0], w["K"][1] + 1))
        gamma = float(rng.uniform(w["gamma"][0], w["gamma"][1]))
        m = max(1, m_from_gamma(gamma, p))
        out.append(dict(n=n, p=p, K=K, gamma=gamma, m=m, seed=i))
    return out


def batch_set_torch(name, i, prm, device="cuda", n=None):
    """Set i of a batched workload drawn with torch on `device` (mixture-style:
    the set's own K centers N(0, 4 I), unit noise, 1% of entries replaced by
    20 t_3)."""
    import torch

    w = WORKLOADS[name]
    n = prm["n"] if n is None else n
    p, K = prm["p"], prm["K"]
    rng = np.random.default_rng([w["data_seed"], 0xCE7, i])
    C = torch.as_tensor(w["center_std"] * rng.standard_normal((K, p)), dtype=torch.float32, device=device)
    g = torch.Generator(device=device)
    g.manual_seed((w["data_seed"] * 1000003 + 23) * 1000003 + i)
    lab = torch.randint(0, K, (n,), generator=g, device=device)
    X = C[lab] + torch.randn((n, p), generator=g, device=device)
    mask = torch.rand((n, p), generator=g, device=device) < w["spike_prob"]
    nsp = int(mask.sum())
    z = torch.randn(nsp, generator=g, device=device)
    chi = torch.zeros(nsp, device=device)
    for _ in range(w["spike_dof"]):
        chi += torch.randn(nsp, generator=g, device=device) ** 2
    X[mask] = w["spike_scale"] * z / torch.sqrt(chi / w["spike_dof"])
    return X
