"""GPU parity: every C-ABI entry point against the FP64 CPU oracle on the same
seeded inputs.

Bars: sampled indices and K-means assignments bit-exact; floating-point
results within a normwise tolerance, max|delta| / max|oracle| (and the
Frobenius ratio for covariances): 1e-12 for FP64 plans (values 1e-13), 1e-5 for
FP32 and split-BF16 plans (values 1e-6).  Sizes span several tiles and splits
with ragged tails.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1511_00152_amd as pds  # noqa: E402
import synth  # noqa: E402
from oracle import ref  # noqa: E402

pytestmark = pytest.mark.gpu

PRECS = {
    "f64": (pds.PDS_F64, np.float64, 1e-13, 1e-12),
    "f32": (pds.PDS_F32, np.float32, 1e-6, 1e-5),
    "split": (pds.PDS_SPLIT_BF16, np.float32, 1e-6, 1e-5),
}


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


def nerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def ferr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def u16(t):
    return t.cpu().numpy().view(np.uint16)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def log(msg):
    print(msg, flush=True)


# ------------------------------------------------------------------ compress --
COMPRESS_SHAPES = [(2, 1, 77), (2, 2, 5), (16, 5, 300), (64, 7, 257), (128, 13, 1000), (256, 26, 1031),
                   (512, 51, 777), (1024, 51, 2049), (2048, 205, 513), (4096, 410, 1500), (8192, 100, 65),
                   (32768, 500, 4), (65536, 300, 3), (256, 256, 100), (1024, 1, 333)]


@pytest.mark.parametrize("prec", list(PRECS))
@pytest.mark.parametrize("p,m,n", COMPRESS_SHAPES)
def test_compress_matches_oracle(p, m, n, prec):
    pr, dt, vtol, _ = PRECS[prec]
    log(f"compress p={p} m={m} n={n} prec={prec}")
    X = np.random.default_rng([p, m, n]).standard_normal((n, p)).astype(dt)
    seed = 7 + p
    plan = pds.Plan(p, m, seed=seed, prec=pr)
    vals, idx = pds.compress(plan, to_dev(X))
    torch.cuda.synchronize()
    v_o, i_o = ref.compress(X, seed, m)
    assert np.array_equal(u16(idx), i_o)
    assert nerr(vals.cpu().numpy().astype(np.float64), v_o) <= vtol


def test_sampler_rejection_path_bit_exact():
    """p = 65536, m = 32768: about one sample in five needs an extra word after
    a Lemire rejection; those rows still match the oracle bit for bit."""
    p, m, n = 65536, 32768, 20
    assert sum(ref.sample_words_used(0, i, p, m) > m for i in range(n)) >= 2
    X = np.random.default_rng(0).standard_normal((n, p)).astype(np.float32)
    plan = pds.Plan(p, m, seed=0, prec=pds.PDS_F32)
    vals, idx = pds.compress(plan, to_dev(X))
    torch.cuda.synchronize()
    v_o, i_o = ref.compress(X, 0, m)
    assert np.array_equal(u16(idx), i_o)
    assert nerr(vals.cpu().numpy().astype(np.float64), v_o) <= 1e-6


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_compress_chunked_equals_one_shot(prec):
    pr, dt, _, _ = PRECS[prec]
    p, m, n = 1024, 51, 3000
    X = to_dev(np.random.default_rng(1).standard_normal((n, p)).astype(dt))
    plan = pds.Plan(p, m, seed=3, prec=pr)
    v1, i1 = pds.compress(plan, X)
    parts = [pds.compress(plan, X[a:b], i0=a) for a, b in [(0, 1000), (1000, 1001), (1001, 3000)]]
    torch.cuda.synchronize()
    assert torch.equal(i1, torch.cat([q[1] for q in parts]))
    assert torch.equal(v1, torch.cat([q[0] for q in parts]))
    v2, i2 = pds.compress(plan, X)
    torch.cuda.synchronize()
    assert torch.equal(v1, v2) and torch.equal(i1, i2)  # deterministic


@pytest.mark.parametrize("p", [256, 1024, 4096])
def test_compress_strided_rows(p):
    """A leading dimension that breaks 16-byte row alignment takes the generic path."""
    m, n = p // 10, 129
    Xb = np.random.default_rng(2).standard_normal((n, p + 1)).astype(np.float32)
    Xt = to_dev(Xb)[:, :p]
    plan = pds.Plan(p, m, seed=1, prec=pds.PDS_F32)
    vals, idx = pds.compress(plan, Xt)
    torch.cuda.synchronize()
    v_o, i_o = ref.compress(np.ascontiguousarray(Xb[:, :p]), 1, m)
    assert np.array_equal(u16(idx), i_o)
    assert nerr(vals.cpu().numpy().astype(np.float64), v_o) <= 1e-6


# Split plans at p = 4096 take the Kronecker matrix-core transform (one wave
# per sample, persistent, the next row and the first 512 kept indices requested
# ahead): fewer samples than waves, m = 1 and 2, m past the 512 requested ahead,
# m = p.
KRON_SHAPES = [(410, 1), (410, 31), (410, 33), (1, 100), (2, 65), (600, 300), (1000, 97), (3840, 40), (4096, 20)]


@pytest.mark.parametrize("m,n", KRON_SHAPES)
def test_split_4096_kron_matches_oracle(m, n):
    p = 4096
    log(f"split p=4096 m={m} n={n}")
    X = np.random.default_rng([m, n]).standard_normal((n, p)).astype(np.float32)
    plan = pds.Plan(p, m, seed=5 + m, prec=pds.PDS_SPLIT_BF16)
    vals, idx = pds.compress(plan, to_dev(X))
    torch.cuda.synchronize()
    v_o, i_o = ref.compress(X, 5 + m, m)
    assert np.array_equal(u16(idx), i_o)
    assert nerr(vals.cpu().numpy().astype(np.float64), v_o) <= 1e-6


def test_split_4096_chunked_equals_one_shot():
    """Chunked calls (i0 > 0, ragged chunk sizes) reproduce a one-shot call bit for bit."""
    p, m, n = 4096, 410, 1000
    X = to_dev(np.random.default_rng(3).standard_normal((n, p)).astype(np.float32))
    plan = pds.Plan(p, m, seed=8, prec=pds.PDS_SPLIT_BF16)
    v1, i1 = pds.compress(plan, X)
    parts = [pds.compress(plan, X[a:b], i0=a) for a, b in [(0, 45), (45, 46), (46, 517), (517, 1000)]]
    torch.cuda.synchronize()
    assert torch.equal(i1, torch.cat([q[1] for q in parts]))
    assert torch.equal(v1, torch.cat([q[0] for q in parts]))


def test_compress_empty_is_noop():
    plan = pds.Plan(256, 26, prec=pds.PDS_F32)
    X = torch.empty((0, 256), dtype=torch.float32, device="cuda")
    vals, idx = pds.compress(plan, X)
    assert vals.shape == (0, 26)


# ---------------------------------------------------------------- covariance --
# the last three run many 32-sample chunks per workgroup (the clear-then-write
# order between chunks), the dense one through the long-run overflow loops
COV_SHAPES = [(2, 2, 50), (16, 4, 33), (64, 7, 1000), (128, 20, 31), (256, 26, 2000), (512, 64, 4099),
              (1024, 51, 20000), (4096, 410, 3000), (8192, 200, 100), (256, 256, 300),
              (256, 26, 40000), (2048, 205, 30000), (1024, 1024, 2000)]


# (precision, Gram form): FP64 plans have the dense form only
GRAM_FORMS = {"dense": pds.PDS_GRAM_DENSE, "sparse": pds.PDS_GRAM_SPARSE}
PREC_GRAM = [("f64", "dense"), ("f32", "dense"), ("f32", "sparse"), ("split", "dense"), ("split", "sparse")]


@pytest.mark.parametrize("prec,gram", PREC_GRAM)
@pytest.mark.parametrize("p,m,n", COV_SHAPES)
def test_covariance_matches_oracle(p, m, n, prec, gram):
    pr, dt, _, tol = PRECS[prec]
    log(f"covariance p={p} m={m} n={n} prec={prec} gram={gram}")
    d = synth.random_compressed(n, p, m, seed=p + m, dtype=dt)
    plan = pds.Plan(p, m, seed=0, prec=pr, gram=GRAM_FORMS[gram])
    C = pds.covariance(plan, to_dev(d["vals"]), to_dev(d["idx"].view(np.int16)))
    torch.cuda.synchronize()
    C_o = ref.covariance(p, d["vals"].astype(np.float64), d["idx"])
    Cg = C.cpu().numpy()
    assert np.array_equal(Cg, Cg.T)
    assert nerr(Cg, C_o) <= tol and ferr(Cg, C_o) <= tol, (nerr(Cg, C_o), ferr(Cg, C_o))


def test_sparse_gram_deterministic_and_scale_changes():
    """The sparse form sums integers: two runs give the same bits.  Values
    whose size changes by 2^20 between fixed-point ranges (2048 samples) and
    super-ranges still meet the bar against the oracle."""
    p, m, n = 1024, 51, 70001
    d = synth.random_compressed(n, p, m, seed=77, dtype=np.float32)
    v = d["vals"]
    scale = np.ones(n, dtype=np.float32)
    scale[5000:9000] = 1024.0
    scale[20000:20100] = 1.0 / 1024.0
    scale[60000] = 2.0 ** 20
    v = (v * scale[:, None]).astype(np.float32)
    plan = pds.Plan(p, m, seed=0, prec=pds.PDS_F32, gram=pds.PDS_GRAM_SPARSE)
    vals, idx = to_dev(v), to_dev(d["idx"].view(np.int16))
    C1 = pds.covariance(plan, vals, idx).cpu().numpy()
    C2 = pds.covariance(plan, vals, idx).cpu().numpy()
    assert np.array_equal(C1, C2)
    C_o = ref.covariance(p, v.astype(np.float64), d["idx"])
    log(f"sparse Gram with scale changes: nerr {nerr(C1, C_o):.3e} ferr {ferr(C1, C_o):.3e}")
    assert nerr(C1, C_o) <= 1e-5 and ferr(C1, C_o) <= 1e-5


def test_sparse_gram_non_finite_value_poisons_its_tiles():
    p, m, n = 512, 40, 3000
    d = synth.random_compressed(n, p, m, seed=5, dtype=np.float32)
    v = d["vals"].copy()
    v[1234, 7] = np.nan
    plan = pds.Plan(p, m, seed=0, prec=pds.PDS_F32, gram=pds.PDS_GRAM_SPARSE)
    C = pds.covariance(plan, to_dev(v), to_dev(d["idx"].view(np.int16))).cpu().numpy()
    j = int(d["idx"][1234, 7])
    assert np.isnan(C[j, j])


@pytest.mark.parametrize("prec,gram", PREC_GRAM)
def test_covariance_streaming_batches(prec, gram):
    pr, dt, _, tol = PRECS[prec]
    p, m, n = 512, 51, 5000
    d = synth.random_compressed(n, p, m, seed=11, dtype=dt)
    plan = pds.Plan(p, m, prec=pr, gram=GRAM_FORMS[gram])
    acc = pds.CovarianceAccumulator(plan)
    vals, idx = to_dev(d["vals"]), to_dev(d["idx"].view(np.int16))
    for a, b in [(0, 1700), (1700, 1701), (1701, 5000)]:
        acc.add(vals[a:b], idx[a:b])
    C = acc.finalize()
    torch.cuda.synchronize()
    C_o = ref.covariance(p, d["vals"].astype(np.float64), d["idx"])
    assert nerr(C.cpu().numpy(), C_o) <= tol


@pytest.mark.parametrize("prec", list(PRECS))
def test_compress_then_covariance_end_to_end(prec):
    """X -> (vals, idx) -> C_n on both sides from the same X bytes."""
    pr, dt, _, tol = PRECS[prec]
    name = "small_f64" if prec == "f64" else "spiked4096_f32"
    w = synth.WORKLOADS[name]
    p = w["p"]
    m = synth.m_from_gamma(w["gamma"], p)
    n = 2000 if prec == "f64" else 4133
    X = synth.rows_numpy(name, n).astype(dt)
    plan = pds.Plan(p, m, seed=0, prec=pr)
    vals, idx = pds.compress(plan, to_dev(X))
    C = pds.covariance(plan, vals, idx)
    torch.cuda.synchronize()
    v_o, i_o = ref.compress(X, 0, m)
    C_o = ref.covariance(p, v_o, i_o)
    assert np.array_equal(u16(idx), i_o)
    Cg = C.cpu().numpy()
    log(f"e2e cov {name} n={n}: nerr {nerr(Cg, C_o):.3e} ferr {ferr(Cg, C_o):.3e}")
    assert nerr(Cg, C_o) <= tol and ferr(Cg, C_o) <= tol
    k = min(20, p)
    ev = np.linalg.eigvalsh(Cg)[::-1][:k]
    ev_o = np.linalg.eigvalsh(C_o)[::-1][:k]
    assert np.max(np.abs(ev - ev_o) / np.abs(ev_o)) <= tol


# ------------------------------------------------------------------- K-means --
# every assignment path: FP32 cooperative (K <= 32), FP32 with LDS sums (K > 32),
# FP32 with global sums (K p beyond LDS), FP64 with LDS sums, FP64 global
KM_PATHS = [("f32", 1024, 51, 10, 20000), ("f32", 128, 13, 40, 9000), ("f32", 2048, 205, 50, 3000),
            ("f64", 256, 26, 5, 7000), ("f64", 1024, 51, 100, 3000)]


@pytest.mark.parametrize("prec,p,m,K,n", KM_PATHS)
def test_kmeans_step_deterministic(prec, p, m, K, n):
    """Every K-means sum is fixed point (exact integers): two calls give the
    same bits, on every assignment path."""
    pr, dt, _, _ = PRECS[prec]
    d = synth.random_compressed(n, p, m, seed=K + p, dtype=dt, K=K)
    plan = pds.Plan(p, m, seed=0, prec=pr)
    vals, idx = to_dev(d["vals"]), to_dev(d["idx"].view(np.int16))
    C0 = to_dev(d["centers"])
    r1 = [t.cpu().numpy().copy() for t in pds.kmeans_step(plan, vals, idx, C0)]
    r2 = [t.cpu().numpy().copy() for t in pds.kmeans_step(plan, vals, idx, C0)]
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b)
    mu_o, a_o, J_o, _ = ref.kmeans_step(p, d["vals"].astype(np.float64), d["idx"], d["centers"])
    assert np.array_equal(r1[1], a_o)
    tol = 1e-12 if prec == "f64" else 1e-5
    assert nerr(r1[0], mu_o) <= tol and abs(float(r1[2][0]) - J_o) <= tol * J_o


@pytest.mark.parametrize("prec,p,m,K,n", KM_PATHS + [("f32", 1024, 100, 10, 20000), ("f64", 4096, 100, 100, 700)])
@pytest.mark.parametrize("T", [1, 2, 5])
def test_kmeans_run_equals_successive_steps(prec, p, m, K, n, T):
    """T rounds in one call (rounds after the first reuse the first round's
    per-workgroup scales) give the bits of T successive kmeans_step calls:
    centers, the last assignments and every round's objective, on every
    assignment path; the centers entering the call stay untouched."""
    pr, dt, _, _ = PRECS[prec]
    d = synth.random_compressed(n, p, m, seed=K + p + T, dtype=dt, K=K)
    plan = pds.Plan(p, m, seed=0, prec=pr)
    vals, idx = to_dev(d["vals"]), to_dev(d["idx"].view(np.int16))
    C0 = to_dev(d["centers"])
    C0_copy = C0.clone()
    C_r, a_r, J_r = pds.kmeans_run(plan, vals, idx, C0, T)
    C = C0
    Js = []
    for _ in range(T):
        C, a, J = pds.kmeans_step(plan, vals, idx, C)
        Js.append(float(J.item()))
    torch.cuda.synchronize()
    assert torch.equal(C_r, C)
    assert torch.equal(a_r, a)
    assert np.array_equal(J_r.cpu().numpy(), np.array(Js))
    assert torch.equal(C0, C0_copy)


KM_SHAPES = [(256, 26, 2000, 5), (1024, 51, 9000, 10), (64, 64, 500, 3), (128, 1, 300, 4), (512, 40, 1000, 1),
             (256, 30, 3000, 37), (4096, 100, 700, 100),
             # FP32 cooperative assignment, one instance per four-cluster group count
             # (a quad per sample for m <= 64, a DPP row beyond)
             (128, 12, 800, 16), (256, 20, 1500, 23), (256, 26, 1200, 32), (256, 65, 1500, 7),
             (512, 100, 3000, 8), (2048, 205, 2000, 20)]


@pytest.mark.parametrize("prec", list(PRECS))
@pytest.mark.parametrize("p,m,n,K", KM_SHAPES)
def test_kmeans_step_matches_oracle(p, m, n, K, prec):
    pr, dt, _, tol = PRECS[prec]
    log(f"kmeans p={p} m={m} n={n} K={K} prec={prec}")
    d = synth.random_compressed(n, p, m, seed=p * 3 + K, dtype=dt, K=K)
    plan = pds.Plan(p, m, prec=pr)
    c_in = d["centers"]
    mu, a, J = pds.kmeans_step(plan, to_dev(d["vals"]), to_dev(d["idx"].view(np.int16)), to_dev(c_in))
    torch.cuda.synchronize()
    mu_o, a_o, J_o, margin = ref.kmeans_step(p, d["vals"].astype(np.float64), d["idx"], c_in)
    ag = a.cpu().numpy()
    assert np.array_equal(ag, a_o), np.nonzero(ag != a_o)[0][:10]
    assert nerr(mu.cpu().numpy(), mu_o) <= tol
    assert abs(J.item() - J_o) <= tol * J_o


# (p, n, K, prec, ld_extra): ragged row counts, ldx > p, one cluster window and several, K > 64
KM2_SHAPES = [(256, 2000, 5, "f64", 0), (1024, 3001, 10, "f32", 0), (64, 777, 3, "split", 4), (4096, 300, 20, "f32", 0),
              (128, 513, 37, "f32", 8), (8, 100, 2, "f64", 0), (512, 1500, 100, "f32", 0), (2, 50, 1, "f32", 0)]


@pytest.mark.parametrize("p,n,K,prec,ld_extra", KM2_SHAPES)
def test_kmeans_2pass_matches_oracle(p, n, K, prec, ld_extra):
    """Second pass of two-pass K-means against the oracle on the same X, one-pass
    assignments (one cluster left empty when K > 2) and centers: assignments
    bit-exact, centers to the FP64 tolerance."""
    pr, dt, _, _ = PRECS[prec]
    log(f"kmeans 2-pass p={p} n={n} K={K} prec={prec}")
    rng = np.random.default_rng([p, n, K])
    means = rng.standard_normal((K, p)) * 2.0
    X = (means[rng.integers(0, K, n)] + rng.standard_normal((n, p))).astype(dt)
    Xl = np.zeros((n, p + ld_extra), dtype=dt)
    Xl[:, :p] = X
    c_hat = rng.integers(0, max(K - 1, 1), n).astype(np.int32) if K > 2 else rng.integers(0, K, n).astype(np.int32)
    mu_hat = means + 0.1 * rng.standard_normal((K, p))
    plan = pds.Plan(p, max(1, p // 10), prec=pr)
    mu, c = pds.kmeans_2pass(plan, to_dev(Xl)[:, :p], to_dev(c_hat), to_dev(mu_hat))
    torch.cuda.synchronize()
    mu_o, c_o, _ = ref.kmeans_2pass(X.astype(np.float64), c_hat, mu_hat)
    cg = c.cpu().numpy()
    assert np.array_equal(cg, c_o), np.nonzero(cg != c_o)[0][:10]
    assert nerr(mu.cpu().numpy(), mu_o) <= 1e-12


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_kmeans_2pass_near_ties_resolved_in_fp64(prec):
    """One-pass centers 1e-9 apart and an exact duplicate: the FP64 recheck
    gives the oracle's argmin, duplicates go to the lower index."""
    pr, dt, _, _ = PRECS[prec]
    p, n, K = 256, 3000, 4
    rng = np.random.default_rng(9)
    X = rng.standard_normal((n, p)).astype(dt)
    mu_hat = rng.standard_normal((K, p)) * 0.5
    mu_hat[1] = mu_hat[0]
    mu_hat[1, 3] += 1e-9
    mu_hat[3] = mu_hat[2]
    c_hat = rng.integers(0, K, n).astype(np.int32)
    plan = pds.Plan(p, 26, prec=pr)
    _, c = pds.kmeans_2pass(plan, to_dev(X), to_dev(c_hat), to_dev(mu_hat))
    torch.cuda.synchronize()
    _, c_o, margin = ref.kmeans_2pass(X.astype(np.float64), c_hat, mu_hat)
    cg = c.cpu().numpy()
    assert np.sum(margin < 1e-6) > 0  # the case does exercise near ties
    assert np.array_equal(cg, c_o)
    assert not np.any(cg == 3)


def test_kmeans_2pass_after_one_pass_pipeline():
    """Alg. 2 on the mixture workload's shape: the oracle's own one-pass run
    gives (c_hat, mu_hat); the GPU second pass equals the oracle's."""
    w = synth.WORKLOADS["mixture_f32"]
    p, K = w["p"], w["K"]
    m = synth.m_from_gamma(w["gamma"], p)
    n = 6000
    X = synth.rows_numpy("mixture_f32", n).astype(np.float32)
    one = ref.sparsified_kmeans(X, 0, m, K, 5)
    plan = pds.Plan(p, m, seed=0, prec=pds.PDS_F32)
    mu, c = pds.kmeans_2pass(plan, to_dev(X), to_dev(one["assign"].astype(np.int32)), to_dev(one["centers"]))
    torch.cuda.synchronize()
    mu_o, c_o, _ = ref.kmeans_2pass(X.astype(np.float64), one["assign"], one["centers"])
    assert np.array_equal(c.cpu().numpy(), c_o)
    assert nerr(mu.cpu().numpy(), mu_o) <= 1e-12


def test_kmeans_2pass_argument_errors():
    plan = pds.Plan(64, 8, prec=pds.PDS_F32)
    X = torch.zeros((10, 64), dtype=torch.float32, device="cuda")
    c = torch.zeros(10, dtype=torch.int32, device="cuda")
    mu = torch.zeros((3, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(pds.PdsError):
        pds.kmeans_2pass(plan, X, c, mu, out=mu)  # aliasing
    with pytest.raises(pds.PdsError):
        X32 = torch.zeros((10, 32), dtype=torch.float32, device="cuda")
        pds.kmeans_2pass(plan, X32, c, mu)  # ldx = 32 < p = 64


@pytest.mark.parametrize("prec", ["f32", "split"])
def test_kmeans_near_ties_resolved_in_fp64(prec):
    """Centers that differ by ~1e-9 relative in one coordinate: FP32 distances
    cannot separate them, the FP64 recheck must give the FP64 argmin; exact
    duplicates must go to the lower index."""
    pr, dt, _, _ = PRECS[prec]
    p, m, n, K = 256, 26, 4000, 4
    d = synth.random_compressed(n, p, m, seed=5, dtype=dt, K=K)
    c = d["centers"].copy()
    c[1] = c[0]
    c[1, 7] += 3e-9       # coordinate 7: samples keeping it prefer one of 0/1 by ~1e-9
    c[3] = c[2]           # exact duplicate: ties go to 2
    plan = pds.Plan(p, m, prec=pr)
    _, a, _ = pds.kmeans_step(plan, to_dev(d["vals"]), to_dev(d["idx"].view(np.int16)), to_dev(c))
    torch.cuda.synchronize()
    _, a_o, _, margin = ref.kmeans_step(p, d["vals"].astype(np.float64), d["idx"], c)
    assert np.any(margin[(a_o == 0) | (a_o == 1)] < 1e-6)
    assert np.array_equal(a.cpu().numpy(), a_o)
    assert not np.any(a.cpu().numpy() == 3)


@pytest.mark.parametrize("prec", list(PRECS))
def test_unmix_matches_oracle(prec):
    pr, _, _, _ = PRECS[prec]
    for p, K in [(2, 1), (256, 5), (1024, 10), (8192, 3)]:
        c = np.random.default_rng(p).standard_normal((K, p))
        plan = pds.Plan(p, 1, seed=9, prec=pr)
        out = pds.unmix(plan, to_dev(c))
        torch.cuda.synchronize()
        assert nerr(out.cpu().numpy(), ref.unmix(9, c)) <= 1e-13


def test_small_config_end_to_end_fp64():
    """The small FP64 workload in full: n=2000, p=256, m=26, K=5, 10 rounds of
    Alg. 1 from the oracle's K-means++ seeding; every round's assignments equal,
    centers and objective within 1e-12, unmixed centers within 1e-12."""
    w = synth.WORKLOADS["small_f64"]
    p, K, T = w["p"], w["K"], w["T"]
    m = synth.m_from_gamma(w["gamma"], p)
    X = synth.rows_numpy("small_f64")
    plan = pds.Plan(p, m, seed=0, prec=pds.PDS_F64)
    vals, idx = pds.compress(plan, to_dev(X))
    v_o, i_o = ref.compress(X, 0, m)
    mu0, _ = ref.kmeanspp(0, p, v_o, i_o, K)
    mu_g = to_dev(mu0)
    mu_o = mu0
    for t in range(T):
        mu_g, a_g, J_g = pds.kmeans_step(plan, vals, idx, mu_g)
        mu_o, a_o, J_o, _ = ref.kmeans_step(p, v_o, i_o, mu_o)
        torch.cuda.synchronize()
        assert np.array_equal(a_g.cpu().numpy(), a_o), t
        assert nerr(mu_g.cpu().numpy(), mu_o) <= 1e-12
        assert abs(J_g.item() - J_o) <= 1e-12 * J_o
    cen = pds.unmix(plan, mu_g)
    torch.cuda.synchronize()
    assert nerr(cen.cpu().numpy(), ref.unmix(0, mu_o)) <= 1e-12


def test_mixture_kmeans_reduced_n_fp32():
    """The FP32 mixture workload (p=1024, K=10, m=51) at n = 2^14 + 37: 20
    rounds from the oracle's seeding, both sides from the same X bytes.  The
    GPU's FP32 compressed values differ from the oracle's FP64 ones by rounding,
    so an assignment may differ only where the oracle's own margin is below the
    FP32 noise of a distance; centers stay within 1e-5."""
    w = synth.WORKLOADS["mixture_f32"]
    p, K, T = w["p"], w["K"], w["T"]
    m = synth.m_from_gamma(w["gamma"], p)
    n = (1 << 14) + 37
    X = synth.rows_numpy("mixture_f32", n)
    plan = pds.Plan(p, m, seed=0, prec=pds.PDS_F32)
    vals, idx = pds.compress(plan, to_dev(X))
    v_o, i_o = ref.compress(X, 0, m)
    mu0, _ = ref.kmeanspp(0, p, v_o, i_o, K)
    mu_g, mu_o = to_dev(mu0), mu0
    for t in range(T):
        mu_g, a_g, J_g = pds.kmeans_step(plan, vals, idx, mu_g)
        mu_o, a_o, J_o, margin = ref.kmeans_step(p, v_o, i_o, mu_o)
        torch.cuda.synchronize()
        bad = np.nonzero(a_g.cpu().numpy() != a_o)[0]
        assert np.all(margin[bad] <= 1e-4 * (J_o / n)), (t, bad[:5], margin[bad][:5])
        assert nerr(mu_g.cpu().numpy(), mu_o) <= 1e-5
        assert abs(J_g.item() - J_o) <= 1e-5 * J_o


# ------------------------------------------------------------- eigenvalues --
@pytest.mark.parametrize("p", [16, 257, 1024])
def test_top_eigenvalues_match_lapack(p):
    """top_eigenvalues (device solver) against LAPACK on the host, for a
    symmetric indefinite matrix and for a covariance estimate of the pipeline."""
    log(f"top_eigenvalues p={p}")
    rng = np.random.default_rng(p)
    A = rng.standard_normal((p, p))
    A = A + A.T
    ev = pds.top_eigenvalues(to_dev(A), 20).cpu().numpy()
    ev_o = np.linalg.eigvalsh(A)[::-1][:min(20, p)]
    assert np.max(np.abs(ev - ev_o)) <= 1e-10 * np.max(np.abs(ev_o))


def test_top_eigenvalues_of_the_estimate():
    p, m, n = 256, 64, 3000
    X = synth.rows_numpy("small_f64", n)
    plan = pds.Plan(p, m, seed=0, prec=pds.PDS_F64)
    vals, idx = pds.compress(plan, to_dev(X))
    C = pds.covariance(plan, vals, idx)
    v_o, i_o = ref.compress(X, 0, m)
    C_o = ref.covariance(p, v_o, i_o)
    ev = pds.top_eigenvalues(C, 20).cpu().numpy()
    ev_o = np.linalg.eigvalsh(C_o)[::-1][:20]
    assert np.max(np.abs(ev - ev_o) / np.abs(ev_o)) < 1e-11
