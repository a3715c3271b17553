"""Parity at the full workload sizes, in the launch configuration bench.py
times.

* p = 4096, n = 2^20, m = 410 (both precision forms): the whole covariance is
  out of the oracle's reach in test time, so the oracle computes a principal
  submatrix C[J][J] over 24 seeded coordinates straight from the definitions
  (every sample's kept set, explicit Hadamard rows for the kept entries of J),
  and 256 sampled rows of (idx, vals) one by one.
* Mixture, p = 1024, n = 2^20, m = 51, K = 10: the oracle runs the whole
  workload (compression, seeding, 20 rounds); assignments may differ only at
  near ties of the oracle's own distances, centers within 1e-5.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1511_00152_amd as pds  # noqa: E402
import synth  # noqa: E402
from oracle import ref  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def nerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def spiked():
    w = synth.WORKLOADS["spiked4096_f32"]
    p, n = w["p"], w["n"]
    m = synth.m_from_gamma(w["gamma"], p)
    X = synth.rows_torch("spiked4096_f32", n, device="cuda")  # the bench's input
    torch.cuda.synchronize()
    print(f"spiked4096 full: n={n} p={p} m={m}", flush=True)
    Xh = X.cpu().numpy()
    J = np.sort(np.random.default_rng(2024).choice(p, 24, replace=False))
    G = ref.gram_submatrix(0, m, Xh, J)
    d = np.diag(G).copy()
    Csub = (p * (p - 1)) / (m * (m - 1)) * G / n
    np.fill_diagonal(Csub, np.diag(Csub) - (p - m) / (p - 1) * np.diag(Csub))
    return {"X": X, "Xh": Xh, "p": p, "m": m, "n": n, "J": J, "Csub": Csub}


@pytest.mark.parametrize("prec", ["split", "f32"])
def test_spiked4096_full_size(spiked, prec):
    p, m, n, J = spiked["p"], spiked["m"], spiked["n"], spiked["J"]
    plan = pds.Plan(p, m, seed=0, prec={"split": pds.PDS_SPLIT_BF16, "f32": pds.PDS_F32}[prec])
    vals, idx = pds.compress(plan, spiked["X"])
    C = pds.covariance(plan, vals, idx)
    torch.cuda.synchronize()
    Cg = C[torch.as_tensor(J, device="cuda")][:, torch.as_tensor(J, device="cuda")].cpu().numpy()
    e = nerr(Cg, spiked["Csub"])
    print(f"{prec}: C[J][J] max rel err {e:.3e}", flush=True)
    assert e <= 1e-5
    rows = np.sort(np.random.default_rng(7).choice(n, 256, replace=False))
    ig = idx[torch.as_tensor(rows, device="cuda")].cpu().numpy().view(np.uint16)
    vg = vals[torch.as_tensor(rows, device="cuda")].cpu().numpy().astype(np.float64)
    for k, r in enumerate(rows):
        v_o, i_o = ref.compress(spiked["Xh"][r:r + 1], 0, m, i0=int(r))
        assert np.array_equal(ig[k], i_o[0]), r
        assert np.max(np.abs(vg[k] - v_o[0])) <= 1e-6 * np.max(np.abs(v_o[0])) * 4


def test_mixture_full_size_kmeans():
    w = synth.WORKLOADS["mixture_f32"]
    p, n, K, T = w["p"], w["n"], w["K"], w["T"]
    m = synth.m_from_gamma(w["gamma"], p)
    X = synth.rows_torch("mixture_f32", n, device="cuda")
    torch.cuda.synchronize()
    print(f"mixture full: n={n} p={p} m={m} K={K} T={T}", flush=True)
    Xh = X.cpu().numpy()
    v_o, i_o = ref.compress(Xh, 0, m)
    mu0, _ = ref.kmeanspp(0, p, v_o, i_o, K)
    plan = pds.Plan(p, m, seed=0, prec=pds.PDS_F32)
    out = pds.sparsified_kmeans(plan, X, torch.from_numpy(mu0).cuda(), T)
    torch.cuda.synchronize()
    assert np.array_equal(out["idx"].cpu().numpy().view(np.uint16), i_o)
    mu_o = mu0
    objs = []
    for _ in range(T):
        mu_o, a_o, J_o, margin = ref.kmeans_step(p, v_o, i_o, mu_o)
        objs.append(J_o)
    a_g = out["assign"].cpu().numpy()
    bad = np.nonzero(a_g != a_o)[0]
    print(f"assignment mismatches after {T} rounds: {len(bad)} of {n}", flush=True)
    assert len(bad) <= n * 1e-4
    assert nerr(out["centers_pre"].cpu().numpy(), mu_o) <= 1e-5
    Jg = out["objectives"].cpu().numpy()
    assert np.max(np.abs(Jg - np.array(objs)) / np.array(objs)) <= 1e-5
    assert nerr(out["centers"].cpu().numpy(), ref.unmix(0, mu_o)) <= 1e-5


def test_mixture_full_size_kmeanspp_and_best_of():
    """K-means++ at the mixture size (n = 2^20, p = 1024, m = 51, K = 10) in the
    launch configuration the bench times: both sides seed from the oracle's
    compressed values rounded to FP32 (the GPU plan's value type), so the
    draws see the same numbers and the chosen samples agree exactly; then the
    best of 3 starts with 2 rounds each against the oracle's."""
    w = synth.WORKLOADS["mixture_f32"]
    p, n, K = w["p"], w["n"], w["K"]
    m = synth.m_from_gamma(w["gamma"], p)
    X = synth.rows_torch("mixture_f32", n, device="cuda").cpu().numpy()
    print(f"mixture full K-means++: n={n} p={p} m={m} K={K}", flush=True)
    v_o, i_o = ref.compress(X, 0, m)
    v32 = v_o.astype(np.float32)
    v64 = v32.astype(np.float64)
    plan = pds.Plan(p, m, seed=0, prec=pds.PDS_F32)
    vals, idx = torch.from_numpy(v32).cuda(), torch.from_numpy(i_o.view(np.int16)).cuda()
    C, ch = pds.kmeanspp(plan, vals, idx, K)
    torch.cuda.synchronize()
    C_o, ch_o = ref.kmeanspp(0, p, v64, i_o, K)
    assert np.array_equal(ch.cpu().numpy(), ch_o)
    assert np.array_equal(C.cpu().numpy(), C_o)
    Cb, ab, objs, best = pds.kmeans_best(plan, vals, idx, K, 2, 3)
    torch.cuda.synchronize()
    o = ref.kmeans_best_compressed(p, v64, i_o, 0, K, 2, 3)
    og = objs.cpu().numpy()
    assert np.max(np.abs(og - o["objectives"]) / o["objectives"]) <= 1e-5
    fin = o["objectives"][:, -1]
    b = int(best.cpu()[0])
    assert b == o["best"] or abs(fin[b] - fin[o["best"]]) <= 2e-5 * fin[o["best"]]
    if b == o["best"]:
        assert np.sum(ab.cpu().numpy() != o["assign"]) == 0
        assert nerr(Cb.cpu().numpy(), o["centers_pre"]) <= 1e-5
