"""GPU parity of DCT plans (preconditioner y = C D x with the orthonormal DCT-II,
Sec. III; the paper's p = 784 runs of Sec. VII) against the FP64 oracle's
compress_dct / unmix_dct and its estimators, on the same seeded inputs.

Bars (derived from the arithmetic): kept indices and FP64 K-means assignments
bit-exact.  In its dense form (p with a prime factor above 7, or p > 2048) the
transform is an FP64 product over p terms, so an FP64 plan's values lie within
4 p u ||x_i|| of the oracle's (u = 2^-53; every |C[j][k]| <= sqrt(2/p), so the
terms of y_j sum in absolute value to at most sqrt(2) ||x_i||, and both sides
round each of p additions).  The FFT form (other p) rounds in each of its at
most log2 p radix stages and in the pre- and post-rotations, a few u ||x_i||
per stage (the usual FFT error analysis, e.g. Higham, Accuracy and Stability
of Numerical Algorithms, ch. 24), which stays under the same bar for every p
>= 2.  An FP32 plan's values are that result rounded once, within 2^-24 |y|
more.  Estimators on top take the bars of the Hadamard plans: 1e-12 (FP64),
1e-5 (FP32, split).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1511_00152_amd as pds  # noqa: E402
import synth  # noqa: E402
from oracle import ref  # noqa: E402

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24
PREC = {"f64": (pds.PDS_F64, np.float64), "f32": (pds.PDS_F32, np.float32), "split": (pds.PDS_SPLIT_BF16, np.float32)}


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


def log(msg):
    print(msg, flush=True)


def nerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def dct_plan(p, m, seed, prec):
    return pds.Plan(p, m, seed=seed, prec=PREC[prec][0], transform=pds.PDS_TRANSFORM_DCT)


def rows(n, p, seed, dtype):
    """Rows with a spread of scales and a few large entries (the data the
    preconditioner is for)."""
    rng = np.random.default_rng([n, p, seed])
    X = rng.standard_normal((n, p)) * np.exp(rng.uniform(-3, 3, size=(n, 1)))
    spikes = rng.random((n, p)) < 0.01
    X[spikes] *= 30.0
    return X.astype(dtype)


def check_values(vals, ovals, X, prec, p):
    """Elementwise: |delta| <= 4 p u ||x_i|| (+ 2^-24 |y| for FP32 values)."""
    xn = np.linalg.norm(X.astype(np.float64), axis=1, keepdims=True)
    d = np.abs(vals.astype(np.float64) - ovals)
    bound = 4 * p * U64 * xn + (U32 * np.abs(ovals) if prec != "f64" else 0.0)
    worst = float(np.max(d / np.maximum(bound, 1e-300))) if d.size else 0.0
    log(f"    values: worst delta / bound = {worst:.3f}")
    assert np.all(d <= bound)


# (p, m, n, prec): non-powers of two, a power of two, the paper's 784, the
# largest p, m = p, m = 1, one row, ragged tiles in both directions.  The FFT
# form takes p = 2^a 3^b 5^c 7^d <= 2048 (every radix: 768 = 2^8 3, 945 =
# 3^3 5 7, 9, the largest 2048, an odd count of samples for the pairing); the
# dense form every other p (4096, 8192, 129, 65, the prime 11, 2058 > 2048).
SHAPES = [(784, 78, 1000, "f32"), (784, 40, 130, "f64"), (784, 784, 65, "f64"), (7, 3, 65, "f64"),
          (100, 37, 1, "f32"), (1000, 100, 257, "f64"), (1024, 51, 300, "f32"), (2, 1, 5, "f64"),
          (4096, 410, 70, "f32"), (784, 80, 64, "split"), (8192, 100, 9, "f32"), (129, 1, 200, "f64"),
          (65, 64, 63, "f32"), (768, 77, 99, "f64"), (945, 94, 101, "f64"), (9, 4, 33, "f64"),
          (2048, 205, 65, "f32"), (2048, 100, 17, "f64"), (11, 5, 40, "f64"), (2058, 200, 21, "f64"),
          (3, 3, 7, "f64"), (5, 2, 3, "f32")]


@pytest.mark.parametrize("p,m,n,prec", SHAPES)
def test_dct_compress_matches_oracle(p, m, n, prec):
    log(f"dct compress p={p} m={m} n={n} {prec}")
    X = rows(n, p, 1, PREC[prec][1])
    plan = dct_plan(p, m, 11, prec)
    vals, idx = pds.compress(plan, to_dev(X))
    torch.cuda.synchronize()
    ov, oi = ref.compress_dct(X, 11, m)
    assert np.array_equal(idx.cpu().numpy().view(np.uint16), oi)
    check_values(vals.cpu().numpy(), ov, X, prec, p)


def test_dct_compress_chunked_equals_one_shot():
    """Chunked calls (i0 > 0) reproduce a one-shot call bit for bit."""
    p, m, n = 784, 60, 700
    X = to_dev(rows(n, p, 2, np.float32))
    plan = dct_plan(p, m, 3, "f32")
    v1, i1 = pds.compress(plan, X)
    parts = [pds.compress(plan, X[a:b], i0=a) for a, b in ((0, 129), (129, 512), (512, 700))]
    torch.cuda.synchronize()
    assert torch.equal(torch.cat([q[1] for q in parts]), i1)
    assert torch.equal(torch.cat([q[0] for q in parts]), v1)


def test_dct_compress_keeps_the_same_sets_as_hadamard():
    """The kept sets depend on (seed, i, p, m) only: a DCT plan and a Hadamard
    plan of one (p, m, seed) keep the same coordinates."""
    p, m, n = 1024, 100, 500
    X = to_dev(rows(n, p, 4, np.float32))
    _, i_d = pds.compress(dct_plan(p, m, 9, "f32"), X)
    _, i_h = pds.compress(pds.Plan(p, m, seed=9), X)
    torch.cuda.synchronize()
    assert torch.equal(i_d, i_h)


@pytest.mark.parametrize("p", [7, 100, 784, 945, 4096])
def test_dct_unmix_matches_oracle_and_inverts(p):
    """unmix = D C^T against the oracle, and at m = p, compress then unmix of
    every row returns the rows.  The unmixing advances its cosines by a
    rotation restarted every 32 terms, so each coefficient carries at most
    about 64 roundings more than the forward table: bound (4p + 128) u ||mu'||
    (twice that plus 4p u for the round trip)."""
    log(f"dct unmix p={p}")
    rng = np.random.default_rng(p)
    K = 5
    cpre = rng.standard_normal((K, p))
    plan = dct_plan(p, p, 21, "f64")
    out = pds.unmix(plan, to_dev(cpre)).cpu().numpy()
    o = ref.unmix_dct(21, cpre)
    bound = (4 * p + 128) * U64 * np.linalg.norm(cpre, axis=1, keepdims=True)
    log(f"    unmix: worst delta / bound = {np.max(np.abs(out - o) / bound):.3f}")
    assert np.all(np.abs(out - o) <= bound)
    n = 37
    X = rows(n, p, 5, np.float64)
    vals, idx = pds.compress(plan, to_dev(X))
    assert np.array_equal(idx.cpu().numpy(), np.tile(np.arange(p), (n, 1)))
    back = pds.unmix(plan, vals).cpu().numpy()
    assert np.all(np.abs(back - X) <= (12 * p + 256) * U64 * np.linalg.norm(X, axis=1, keepdims=True))


@pytest.mark.parametrize("prec,gram", [("f64", "dense"), ("f32", "dense"), ("f32", "sparse"), ("split", "dense")])
def test_dct_covariance_matches_oracle(prec, gram):
    """C_n of a DCT plan (p = 784: the Gram runs over 1024 coordinates, the
    extra ones never kept) against the oracle's estimator on its own DCT
    compression."""
    p, m, n = 784, 100, 3001
    log(f"dct covariance {prec} {gram}")
    X = rows(n, p, 6, PREC[prec][1])
    plan = pds.Plan(p, m, seed=13, prec=PREC[prec][0], transform=pds.PDS_TRANSFORM_DCT,
                    gram=pds.PDS_GRAM_DENSE if gram == "dense" else pds.PDS_GRAM_SPARSE)
    vals, idx = pds.compress(plan, to_dev(X))
    C = pds.covariance(plan, vals, idx).cpu().numpy()
    ov, oi = ref.compress_dct(X, 13, m)
    Co = ref.covariance(p, ov, oi)
    tol = 1e-12 if prec == "f64" else 1e-5
    e = nerr(C, Co)
    log(f"    max rel {e:.2e}")
    assert e <= tol
    assert np.array_equal(C, C.T)


def test_dct_sample_mean_matches_oracle():
    p, m, n = 784, 50, 2000
    X = rows(n, p, 7, np.float64)
    plan = dct_plan(p, m, 17, "f64")
    vals, idx = pds.compress(plan, to_dev(X))
    mu = pds.sample_mean(plan, vals, idx).cpu().numpy()
    ov, oi = ref.compress_dct(X, 17, m)
    assert nerr(mu, ref.mean_estimate(p, ov, oi)) <= 1e-12


def test_dct_kmeans_pipeline_fp64():
    """Sec. VII's use of the DCT, at p = 784 in FP64: compression, K-means++
    seeding, 8 rounds and the unmixing, every step against the oracle's chain
    on its own DCT compression; assignments bit-exact in every round."""
    p, m, n, K, T = 784, 78, 4000, 10, 8
    w_rng = np.random.default_rng(31)
    centers = w_rng.standard_normal((K, p)) * 3.0
    lab = w_rng.integers(0, K, size=n)
    X = centers[lab] + w_rng.standard_normal((n, p))
    plan = dct_plan(p, m, 41, "f64")
    vals, idx = pds.compress(plan, to_dev(X))
    ov, oi = ref.compress_dct(X, 41, m)
    C_g, ch_g = pds.kmeanspp(plan, vals, idx, K)
    C_o, ch_o = ref.kmeanspp(41, p, ov, oi, K)
    torch.cuda.synchronize()
    assert np.array_equal(ch_g.cpu().numpy(), ch_o)
    assert nerr(C_g.cpu().numpy(), C_o) <= 1e-12
    for t in range(T):
        C_g, a_g, J_g = pds.kmeans_step(plan, vals, idx, C_g)
        C_o, a_o, J_o, _ = ref.kmeans_step(p, ov, oi, C_o)
        torch.cuda.synchronize()
        assert np.array_equal(a_g.cpu().numpy(), a_o), t
        assert nerr(C_g.cpu().numpy(), C_o) <= 1e-12
        assert abs(J_g.item() - J_o) <= 1e-12 * J_o
    mu = pds.unmix(plan, C_g).cpu().numpy()
    assert nerr(mu, ref.unmix_dct(41, C_o)) <= 1e-12


def test_dct_mnist_size_fp32():
    """The size the paper runs the DCT at (n = 70000 samples of p = 784, here
    seeded synthetic rows of that shape, gamma = 0.1): every row's kept
    indices bit-exact and values within the bound, in the launch configuration
    of a single call."""
    p, m, n = 784, 78, 70000
    X = rows(n, p, 8, np.float32)
    plan = dct_plan(p, m, 0, "f32")
    vals, idx = pds.compress(plan, to_dev(X))
    torch.cuda.synchronize()
    ov, oi = ref.compress_dct(X, 0, m)
    assert np.array_equal(idx.cpu().numpy().view(np.uint16), oi)
    check_values(vals.cpu().numpy(), ov, X, "f32", p)
