"""K-means++ seeding on the GPU (Alg. 1 seeds with K-means++; D^2 sampling
with the sparsified distance of Sec. VI) against the oracle.

Both sides draw the same uniforms and compute the same FP64 distances (same
order, fused multiply-adds), so the chosen samples agree unless a draw lands
within rounding of a boundary of the running sum, which the GPU forms per
block of samples: a differing choice is accepted only there (the test then
checks it against the sequential running sum from numpy and stops comparing,
since later draws depend on it).  Centers are copies of the chosen samples and
compare exactly.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1511_00152_amd as pds  # noqa: E402
import synth  # noqa: E402
from oracle import ref  # noqa: E402

pytestmark = pytest.mark.gpu

U_RND = 2.0 ** -53
PRECS = {"f64": (pds.PDS_F64, np.float64), "f32": (pds.PDS_F32, np.float32), "split": (pds.PDS_SPLIT_BF16, np.float32)}


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def log(msg):
    print(msg, flush=True)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def uniform(seed, k, r=0):
    w = ref.philox4x64_10([k // 4, r, 2, 0], [seed, 0])[k % 4]
    return float(int(w) >> 11) * 2.0 ** -53


def sparse_d2(vals, idx, centers):
    """D^2 of every sample to the nearest of the given zero-filled centers."""
    d = np.full(vals.shape[0], np.inf)
    for c in centers:
        d = np.minimum(d, np.sum((vals - c[idx.astype(np.int64)]) ** 2, axis=1))
    return d


def check_seeding(seed, vals, idx, K, centers_g, chosen_g, r=0):
    n = vals.shape[0]
    C_o, ch_o = ref.kmeanspp(seed, centers_g.shape[1], vals, idx, K, r)
    for k in range(K):
        if chosen_g[k] != ch_o[k]:
            assert k > 0, "the first center is u n and cannot differ"
            d2 = sparse_d2(vals, idx, C_o[:k])
            run = np.cumsum(d2)
            target = uniform(seed, k, r) * run[-1]
            slack = 4 * n * U_RND * run[-1]
            c = int(chosen_g[k])
            lo = run[c - 1] if c > 0 else 0.0
            assert lo - slack <= target < run[c] + slack, (k, c, int(ch_o[k]))
            log(f"draw {k} within rounding of a boundary: GPU {c}, oracle {int(ch_o[k])}")
            return k
        assert np.array_equal(centers_g[k], C_o[k])
    return K


KMPP_CASES = [(2, 1, 50, 3, "f64"), (64, 7, 1000, 5, "f64"), (256, 26, 5000, 10, "f32"), (1024, 51, 20000, 10, "f32"),
              (4096, 410, 3000, 20, "split"), (16384, 100, 600, 8, "f32"), (128, 13, 1, 1, "f64"),
              (256, 26, 257, 300, "f32"), (512, 51, 70001, 37, "f32")]


@pytest.mark.parametrize("p,m,n,K,prec", KMPP_CASES)
def test_kmeanspp_matches_oracle(p, m, n, K, prec):
    pr, dt = PRECS[prec]
    log(f"kmeanspp p={p} m={m} n={n} K={K} prec={prec}")
    d = synth.random_compressed(n, p, m, seed=7 * p + K, dtype=dt)
    seed = 1000 + K
    plan = pds.Plan(p, m, seed=seed, prec=pr)
    C, ch = pds.kmeanspp(plan, to_dev(d["vals"]), to_dev(d["idx"].view(np.int16)), K)
    torch.cuda.synchronize()
    upto = check_seeding(seed, d["vals"].astype(np.float64), d["idx"], K, C.cpu().numpy(), ch.cpu().numpy())
    assert upto >= min(K, 1)


def test_kmeanspp_pipeline_matches_oracle():
    """The mixture workload's shape at reduced n, FP64 plan: GPU compress and
    GPU K-means++ against the oracle's compress and seeding of the same rows
    (the preconditioned values agree to FP64 rounding, so the draws do)."""
    w = synth.WORKLOADS["mixture_f32"]
    p, K = w["p"], w["K"]
    m = synth.m_from_gamma(w["gamma"], p)
    n = 20000
    X = synth.rows_numpy("mixture_f32", n).astype(np.float64)
    log(f"kmeanspp pipeline p={p} m={m} n={n} K={K}")
    plan = pds.Plan(p, m, seed=0, prec=pds.PDS_F64)
    vals, idx = pds.compress(plan, to_dev(X))
    C, ch = pds.kmeanspp(plan, vals, idx, K)
    torch.cuda.synchronize()
    ov, oi = ref.compress(X, 0, m)
    assert np.array_equal(idx.cpu().numpy().view(np.uint16), oi)
    C_o, ch_o = ref.kmeanspp(0, p, ov, oi, K)
    assert np.array_equal(ch.cpu().numpy(), ch_o)
    assert np.max(np.abs(C.cpu().numpy() - C_o)) <= 1e-13 * np.max(np.abs(C_o))


@pytest.mark.parametrize("r", [1, 5, 1023])
def test_kmeanspp_replicates_match_oracle(r):
    p, m, n, K = 512, 51, 6000, 12
    log(f"kmeanspp replicate {r}")
    d = synth.random_compressed(n, p, m, seed=99, dtype=np.float32)
    plan = pds.Plan(p, m, seed=8, prec=pds.PDS_F32)
    C, ch = pds.kmeanspp(plan, to_dev(d["vals"]), to_dev(d["idx"].view(np.int16)), K, replicate=r)
    torch.cuda.synchronize()
    assert check_seeding(8, d["vals"].astype(np.float64), d["idx"], K, C.cpu().numpy(), ch.cpu().numpy(), r) >= 1


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_kmeans_best_of_r_matches_oracle(prec):
    """Best of R starting points on one compression (mixture shape, reduced
    n): the same kept start, per-start objectives, final centers and
    assignments as the oracle's.  FP64: GPU compress against the oracle's
    compress of the same rows.  FP32: both sides take the oracle's compressed
    values rounded to FP32 (so the seeding draws see the same numbers);
    objectives to FP32 rounding of the distances, and the kept start must
    agree unless two starts end within that rounding of each other."""
    pr, dt = {"f64": (pds.PDS_F64, np.float64), "f32": (pds.PDS_F32, np.float32)}[prec]
    w = synth.WORKLOADS["mixture_f32"]
    p, K = w["p"], w["K"]
    m = synth.m_from_gamma(w["gamma"], p)
    n, T, R = 6000, 5, 6
    X = synth.rows_numpy("mixture_f32", n).astype(np.float64)
    log(f"kmeans best-of-{R} p={p} m={m} n={n} K={K} T={T} prec={prec}")
    plan = pds.Plan(p, m, seed=2, prec=pr)
    if prec == "f64":
        vals, idx = pds.compress(plan, to_dev(X))
        o = ref.sparsified_kmeans_best(X, 2, m, K, T, R)
    else:
        ov, oi = ref.compress(X, 2, m)
        v32 = ov.astype(np.float32)
        vals, idx = to_dev(v32), to_dev(oi.view(np.int16))
        o = ref.kmeans_best_compressed(p, v32.astype(np.float64), oi, 2, K, T, R)
    C, a, objs, best = pds.kmeans_best(plan, vals, idx, K, T, R)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == "f64" else 1e-5
    og = objs.cpu().numpy()
    assert np.max(np.abs(og - o["objectives"]) / o["objectives"]) <= tol
    final = o["objectives"][:, -1]
    b = int(best.cpu()[0])
    if b != o["best"]:
        assert prec == "f32" and abs(final[b] - final[o["best"]]) <= 2 * tol * final[o["best"]], (b, o["best"])
        return
    assert np.array_equal(a.cpu().numpy(), o["assign"])
    assert np.max(np.abs(C.cpu().numpy() - o["centers_pre"])) <= tol * np.max(np.abs(o["centers_pre"]))


def test_sparsified_kmeans_seeds_on_the_device():
    """The end-to-end call with K instead of centers: K-means++ on the device
    (one start, and best of 3), against the oracle's Alg. 1 with the same
    seeding (FP64 plan, so both sides see the same compressed values)."""
    w = synth.WORKLOADS["small_f64"]
    p, n, K = w["p"], w["n"], w["K"]
    m = synth.m_from_gamma(w["gamma"], p)
    X = synth.rows_numpy("small_f64", n)
    log(f"sparsified_kmeans with device seeding p={p} m={m} n={n} K={K}")
    plan = pds.Plan(p, m, seed=3, prec=pds.PDS_F64)
    out = pds.sparsified_kmeans(plan, to_dev(X), K, 6)
    torch.cuda.synchronize()
    o = ref.sparsified_kmeans(X, 3, m, K, 6)
    assert np.array_equal(out["assign"].cpu().numpy(), o["assign"])
    assert np.max(np.abs(out["centers"].cpu().numpy() - o["centers"])) <= 1e-12 * np.max(np.abs(o["centers"]))
    out3 = pds.sparsified_kmeans(plan, to_dev(X), K, 6, starts=3)
    torch.cuda.synchronize()
    o3 = ref.sparsified_kmeans_best(X, 3, m, K, 6, 3)
    assert int(out3["best"].cpu()[0]) == o3["best"]
    assert np.array_equal(out3["assign"].cpu().numpy(), o3["assign"])
    assert np.max(np.abs(out3["centers"].cpu().numpy() - o3["centers"])) <= 1e-12 * np.max(np.abs(o3["centers"]))


def test_kmeanspp_argument_errors():
    plan = pds.Plan(64, 8, prec=pds.PDS_F32)
    vals = torch.zeros((10, 8), dtype=torch.float32, device="cuda")
    idx = torch.zeros((10, 8), dtype=torch.int16, device="cuda")
    with pytest.raises(pds.PdsError):
        pds.kmeanspp(plan, vals, idx, 0)
    with pytest.raises(pds.PdsError):
        pds.kmeanspp(plan, vals, idx, 1025)
    with pytest.raises(pds.PdsError):
        pds.kmeanspp(plan, vals[:0], idx[:0], 3)
    with pytest.raises(pds.PdsError):
        pds.kmeanspp(plan, vals, idx, 3, ws=torch.empty(8, dtype=torch.uint8, device="cuda"))
    with pytest.raises(pds.PdsError):
        pds.kmeanspp(plan, vals, idx, 3, replicate=-1)
    with pytest.raises(pds.PdsError):
        pds.kmeans_best(plan, vals, idx, 3, 0, 2)
    with pytest.raises(pds.PdsError):
        pds.kmeans_best(plan, vals, idx, 3, 2, 0)
