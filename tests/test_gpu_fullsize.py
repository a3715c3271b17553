"""Parity at the full workload sizes, in the launch configuration bench.py
times.

* p = 4096, n = 2^20, m = 410 (both precision forms of the metric's
  workload): the oracle compresses all 2^20 rows and sums 256 full rows of
  G = sum_i w_i w_i^T (eight coordinates of every 128-coordinate block, so
  every output tile of the Gram kernels is covered), each entry in sample
  order; the GPU's C_n rows must match within 1e-5 (max and Frobenius,
  normwise).  The kept indices of every row are compared bit for bit and the
  values of every row within the transform's rounding.
* Mixture, p = 1024, n = 2^20, m = 51 (FP32 at scale): the covariance rows the
  same way (32 coordinates per 128-coordinate block); 20 K-means rounds on the
  oracle's compressed values rounded to FP32 (the plan's value type, so both
  sides read identical numbers) with zero assignment mismatches in every
  round; and the pipeline the bench times (GPU compression, then the rounds)
  against the oracle's objectives and centers.
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


def ferr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rows_per_block(p, per_block, seed):
    """`per_block` distinct coordinates of every 128-coordinate block, sorted."""
    rng = np.random.default_rng(seed)
    return np.sort(np.concatenate([b * 128 + rng.choice(128, per_block, replace=False) for b in range(p // 128)]))


def oracle_workload(name, per_block, seed):
    w = synth.WORKLOADS[name]
    p, n = w["p"], w["n"]
    m = synth.m_from_gamma(w["gamma"], p)
    X = synth.rows_torch(name, n, device="cuda")  # the bench's input
    torch.cuda.synchronize()
    print(f"{name} full: n={n} p={p} m={m}; oracle compression of every row", flush=True)
    Xh = X.cpu().numpy()
    v_o, i_o = ref.compress(Xh, 0, m)
    J = rows_per_block(p, per_block, seed)
    print(f"{name}: oracle rows of G ({len(J)} rows)", flush=True)
    C_rows = ref.cov_rows(p, m, n, ref.gram_rows(p, v_o, i_o, J), J)
    return {"X": X, "Xh": Xh, "p": p, "m": m, "n": n, "J": J, "C_rows": C_rows, "v_o": v_o, "i_o": i_o, "w": w}


@pytest.fixture(scope="module")
def spiked():
    return oracle_workload("spiked4096_f32", 8, 2024)


@pytest.fixture(scope="module")
def mixture():
    return oracle_workload("mixture_f32", 32, 2025)


def check_compressed_rows(vals, idx, v_o, i_o):
    """Every row: indices bit-exact, values within 4e-6 of the row's largest
    |value| (FP32 transform of length p: at most log2 p roundings of sums of
    terms no larger than the row's norm)."""
    ig = idx.cpu().numpy().view(np.uint16)
    assert np.array_equal(ig, i_o), f"{int(np.sum(np.any(ig != i_o, axis=1)))} rows with differing indices"
    vg = vals.cpu().numpy().astype(np.float64)
    d = np.max(np.abs(vg - v_o), axis=1)
    s = np.max(np.abs(v_o), axis=1)
    worst = float(np.max(d / np.maximum(s, 1e-300)))
    print(f"values: worst row error {worst:.3e}", flush=True)
    assert worst <= 4e-6


def check_cov_rows(C, wl, tag):
    Jd = torch.as_tensor(wl["J"], device="cuda")
    Cg = C[Jd].cpu().numpy()
    e, f = nerr(Cg, wl["C_rows"]), ferr(Cg, wl["C_rows"])
    print(f"{tag}: {len(wl['J'])} full rows of C_n: max rel err {e:.3e}, Frobenius rel err {f:.3e}", flush=True)
    assert e <= 1e-5 and f <= 1e-5


GRAM = {"dense": pds.PDS_GRAM_DENSE, "sparse": pds.PDS_GRAM_SPARSE}
PRECS = {"split": pds.PDS_SPLIT_BF16, "f32": pds.PDS_F32}


@pytest.mark.parametrize("prec,gram", [("split", "dense"), ("f32", "dense"), ("f32", "sparse"), ("split", "sparse")])
def test_spiked4096_full_size(spiked, prec, gram):
    p, m = spiked["p"], spiked["m"]
    plan = pds.Plan(p, m, seed=0, prec=PRECS[prec], gram=GRAM[gram])
    vals, idx = pds.compress(plan, spiked["X"])
    C = pds.covariance(plan, vals, idx)
    torch.cuda.synchronize()
    check_cov_rows(C, spiked, f"spiked4096 {prec} {gram}")
    check_compressed_rows(vals, idx, spiked["v_o"], spiked["i_o"])


@pytest.mark.parametrize("gram", ["dense", "sparse"])
def test_mixture_full_size_covariance(mixture, gram):
    plan = pds.Plan(mixture["p"], mixture["m"], seed=0, prec=pds.PDS_F32, gram=GRAM[gram])
    vals, idx = pds.compress(plan, mixture["X"])
    C = pds.covariance(plan, vals, idx)
    torch.cuda.synchronize()
    check_cov_rows(C, mixture, f"mixture f32 {gram}")
    check_compressed_rows(vals, idx, mixture["v_o"], mixture["i_o"])


def test_mixture_full_size_kmeans_identical_inputs(mixture):
    """20 rounds from the oracle's K-means++ centers on identical FP32 values:
    the GPU's FP32 distances with the FP64 recheck of near ties must give the
    oracle's FP64 argmin for every sample in every round."""
    p, n, K, T = mixture["p"], mixture["n"], mixture["w"]["K"], mixture["w"]["T"]
    v32 = mixture["v_o"].astype(np.float32)
    v64 = v32.astype(np.float64)
    i_o = mixture["i_o"]
    mu0, _ = ref.kmeanspp(0, p, v64, i_o, K)
    plan = pds.Plan(p, mixture["m"], seed=0, prec=pds.PDS_F32)
    vals, idx = torch.from_numpy(v32).cuda(), torch.from_numpy(i_o.view(np.int16)).cuda()
    ws = plan.workspace(pds.PDS_OP_KMEANS, n, K, device="cuda")
    a_g = torch.from_numpy(mu0).cuda()
    b_g = torch.empty_like(a_g)
    asg = torch.empty(n, dtype=torch.int32, device="cuda")
    obj = torch.empty(1, dtype=torch.float64, device="cuda")
    mu_o = mu0
    for t in range(T):
        pds.kmeans_step(plan, vals, idx, a_g, out=b_g, assign=asg, objective=obj, ws=ws)
        a_g, b_g = b_g, a_g
        mu_o, a_o, J_o, margin = ref.kmeans_step(p, v64, i_o, mu_o)
        bad = np.nonzero(asg.cpu().numpy() != a_o)[0]
        ec = nerr(a_g.cpu().numpy(), mu_o)
        eJ = abs(float(obj.item()) - J_o) / J_o
        print(f"round {t}: {len(bad)} assignment mismatches of {n}; centers {ec:.2e}, objective {eJ:.2e}",
              flush=True)
        assert len(bad) == 0, f"round {t}: oracle margins of the mismatches {margin[bad][:8]}"
        assert ec <= 1e-5 and eJ <= 1e-5


def test_mixture_full_size_kmeans_run_equals_steps(mixture):
    """At the mixture size the 20 rounds of one kmeans_run call (rounds after
    the first reuse the per-workgroup scales of the first) give the bits of 20
    kmeans_step calls: centers, last assignments, every objective."""
    p, n, K, T = mixture["p"], mixture["n"], mixture["w"]["K"], mixture["w"]["T"]
    v32 = mixture["v_o"].astype(np.float32)
    i_o = mixture["i_o"]
    mu0, _ = ref.kmeanspp(0, p, v32.astype(np.float64), i_o, K)
    plan = pds.Plan(p, mixture["m"], seed=0, prec=pds.PDS_F32)
    vals, idx = torch.from_numpy(v32).cuda(), torch.from_numpy(i_o.view(np.int16)).cuda()
    C0 = torch.from_numpy(mu0).cuda()
    C_r, a_r, J_r = pds.kmeans_run(plan, vals, idx, C0, T)
    C, Js = C0, []
    for _ in range(T):
        C, a, J = pds.kmeans_step(plan, vals, idx, C)
        Js.append(float(J.item()))
    torch.cuda.synchronize()
    assert torch.equal(C_r, C) and torch.equal(a_r, a)
    assert np.array_equal(J_r.cpu().numpy(), np.array(Js))


def test_mixture_full_size_kmeans_pipeline(mixture):
    """The bench's pipeline: GPU compression, then 20 rounds from the oracle's
    K-means++ centers; objectives and final centers against the oracle's run
    on its own FP64 compression."""
    p, n, K, T = mixture["p"], mixture["n"], mixture["w"]["K"], mixture["w"]["T"]
    v_o, i_o = mixture["v_o"], mixture["i_o"]
    mu0, _ = ref.kmeanspp(0, p, v_o, i_o, K)
    plan = pds.Plan(p, mixture["m"], seed=0, prec=pds.PDS_F32)
    out = pds.sparsified_kmeans(plan, mixture["X"], torch.from_numpy(mu0).cuda(), T)
    torch.cuda.synchronize()
    assert np.array_equal(out["idx"].cpu().numpy().view(np.uint16), i_o)
    mu_o = mu0
    objs = []
    for _ in range(T):
        mu_o, a_o, J_o, _ = ref.kmeans_step(p, v_o, i_o, mu_o)
        objs.append(J_o)
    Jg = out["objectives"].cpu().numpy()
    eJ = float(np.max(np.abs(Jg - np.array(objs)) / np.array(objs)))
    ec = nerr(out["centers_pre"].cpu().numpy(), mu_o)
    eu = nerr(out["centers"].cpu().numpy(), ref.unmix(0, mu_o))
    print(f"pipeline: objectives {eJ:.2e}, centers {ec:.2e}, unmixed {eu:.2e}", flush=True)
    assert eJ <= 1e-5 and ec <= 1e-5 and eu <= 1e-5


def test_mixture_full_size_kmeanspp_and_best_of(mixture):
    """K-means++ at the mixture size (n = 2^20, p = 1024, m = 51, K = 10) in the
    launch configuration the bench times: both sides seed from the oracle's
    compressed values rounded to FP32 (the GPU plan's value type), so the
    draws see the same numbers and the chosen samples agree exactly; then the
    best of 3 starts with 2 rounds each against the oracle's."""
    p, n, K = mixture["p"], mixture["n"], mixture["w"]["K"]
    i_o = mixture["i_o"]
    v32 = mixture["v_o"].astype(np.float32)
    v64 = v32.astype(np.float64)
    plan = pds.Plan(p, mixture["m"], seed=0, prec=pds.PDS_F32)
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
