"""PCA quality on the GPU against the oracle: the fraction of explained
variance (Sec. II) and principal components of the covariance estimate
(Sec. V).

Explained-variance sums: both sides compute the dots d_ij = x_i . u_j in FP64
(each within p u sum_c |x_ic u_jc| of the exact value, u = 2^-53) and add
n k squares (relative error at most n k u), so the numerators differ by at
most 4 p u sum_ij |d_ij| (|x_i| . |u_j|) + 2 n k u num, the denominators by
2 n p u den.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1511_00152_amd as pds  # noqa: E402
import synth  # noqa: E402
from oracle import ref  # noqa: E402

pytestmark = pytest.mark.gpu

U_RND = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def log(msg):
    print(msg, flush=True)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def orthonormal_rows(rng, k, p):
    Q, _ = np.linalg.qr(rng.standard_normal((p, k)))
    return np.ascontiguousarray(Q.T)


EV_CASES = [(1, 2, 1, "f32", 0), (63, 31, 5, "f64", 0), (64, 64, 16, "f32", 3), (65, 256, 17, "f32", 0),
            (1000, 100, 32, "f64", 5), (4097, 512, 20, "f32", 0), (300, 4096, 20, "f32", 0),
            (70000, 64, 8, "f32", 0)]


@pytest.mark.parametrize("n,p,k,dt,ld_extra", EV_CASES)
def test_explained_variance_matches_oracle(n, p, k, dt, ld_extra):
    log(f"explained_variance n={n} p={p} k={k} {dt} ld+{ld_extra}")
    rng = np.random.default_rng([n, p, k])
    npdt = np.float32 if dt == "f32" else np.float64
    X = (rng.standard_normal((n, p + ld_extra)) * rng.uniform(0.2, 3.0, p + ld_extra)).astype(npdt)
    U = orthonormal_rows(rng, k, p)
    Xd = to_dev(X)[:, :p]
    out = pds.explained_variance(Xd, to_dev(U)).cpu().numpy()
    Xs = X[:, :p].astype(np.float64)
    D = Xs @ U.T
    A = np.abs(Xs) @ np.abs(U).T
    num = float(np.sum(D * D))
    den = float(np.sum(Xs * Xs))
    bnum = 4 * p * U_RND * float(np.sum(np.abs(D) * A)) + 2 * n * k * U_RND * num + 1e-300
    bden = 2 * n * p * U_RND * den
    assert abs(out[0] - num) <= bnum, (out[0], num, bnum)
    assert abs(out[1] - den) <= bden, (out[1], den, bden)
    frac = out[0] / out[1]
    assert abs(frac - ref.explained_variance(Xs, U.T)) <= (bnum / num + bden / den + 4 * U_RND) * frac


def test_explained_variance_full_basis_is_one():
    p, n = 128, 3000
    rng = np.random.default_rng(7)
    X = rng.standard_normal((n, p)).astype(np.float32)
    U = orthonormal_rows(rng, p, p)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    acc = 0.0
    for j0 in range(0, p, 32):  # k is at most 32 per call: add the blocks
        pds.explained_variance(to_dev(X), to_dev(U[j0:j0 + 32]), out=out)
        acc += float(out[0])
    assert abs(acc / float(out[1]) - 1.0) < 1e-12


def test_explained_variance_argument_errors():
    X = torch.zeros((4, 8), dtype=torch.float32, device="cuda")
    U = torch.zeros((33, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(pds.PdsError):
        pds.explained_variance(X, U)  # k = 33 > 32
    with pytest.raises(pds.PdsError):
        pds.explained_variance(X, U[:2], ws=torch.empty(100, dtype=torch.uint8, device="cuda"))
    with pytest.raises(pds.PdsError):
        pds.explained_variance(X[:0], U[:2])  # n = 0


@pytest.mark.parametrize("prec", ["f64", "f32", "split"])
def test_pca_pipeline_matches_oracle(prec):
    """Small workload (p = 256, n = 2000, five planted components): GPU
    compress, covariance, top-5 components and explained variance against the
    oracle's.  The estimates C differ by rounding only; by Davis-Kahan the
    top-k subspaces then differ by sin(theta) <= ||dC||_2 / (gap - ||dC||_2)
    (gap = distance of the 5th from the 6th eigenvalue of the oracle's
    estimate); the projectors then differ by at most 2 k sin(theta) in trace
    norm, so the fraction moves by at most 2 k sin(theta) ||X||_2^2 / ||X||_F^2.
    Eigenvalues move by at most ||dC||_2 (Weyl)."""
    pr, dt = {"f64": (pds.PDS_F64, np.float64), "f32": (pds.PDS_F32, np.float32),
              "split": (pds.PDS_SPLIT_BF16, np.float32)}[prec]
    w = synth.WORKLOADS["small_f64"]
    p, n, k = w["p"], w["n"], 5
    m = synth.m_from_gamma(w["gamma"], p)
    X = synth.rows_numpy("small_f64", n).astype(dt)
    log(f"pca pipeline p={p} m={m} n={n} prec={prec}")
    plan = pds.Plan(p, m, seed=6, prec=pr)
    Xd = to_dev(X)
    vals, idx = pds.compress(plan, Xd)
    C = pds.covariance(plan, vals, idx)
    comps, lam = pds.principal_components(plan, C, k)
    ev = pds.explained_variance(Xd, comps).cpu().numpy()
    ov, oi = ref.compress(X, 6, m)
    C_o = ref.covariance(p, ov, oi)
    U_o = ref.principal_components(C_o, k)
    comps_o = ref.unmix(6, U_o.T)
    ev_o = ref.explained_variance(X.astype(np.float64), comps_o.T)
    w_o = np.sort(np.linalg.eigvalsh(C_o))[::-1]
    dC = np.linalg.norm(C.cpu().numpy() - C_o, 2)
    gap = w_o[k - 1] - w_o[k]
    assert gap > 10 * dC
    assert np.allclose(comps.cpu().numpy() @ comps.cpu().numpy().T, np.eye(k), atol=1e-12)
    assert np.max(np.abs(lam.cpu().numpy() - w_o[:k])) <= dC * (1 + 1e-9) + 1e-12 * w_o[0]
    X64 = X.astype(np.float64)
    sens = 2 * k * np.linalg.norm(X64, 2) ** 2 / np.sum(X64 * X64)
    assert abs(ev[0] / ev[1] - ev_o) <= sens * dC / (gap - dC) + 1e-12
