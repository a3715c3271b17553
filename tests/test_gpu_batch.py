"""GPU parity of the batched form (pds_batch_*) against the FP64 oracle, set by
set: each set's kept coordinates bit-exact, values 1e-6 normwise; K-means
rounds from the same seeding rule (first K compressed samples, zero-filled)
with assignments bit-exact and centers / objectives 1e-5.  The oracle
compresses and clusters from X on its own; nothing it reads comes from the GPU.
Graph replays are checked against the oracle and against each other, with
eager single-set calls in between.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1511_00152_amd as pds  # noqa: E402
from paper_1511_00152_amd import _lib  # noqa: E402
from paper_1511_00152_amd.batch import Batch  # noqa: E402
from oracle import ref  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

# (p, n, m, K, seed, ld_extra)
SETS = [(128, 300, 13, 3, 1, 0), (256, 65, 26, 5, 2, 4), (512, 1, 51, 2, 3, 0), (1024, 1000, 102, 10, 4, 0),
        (2048, 200, 205, 7, 5, 0), (256, 0, 10, 3, 6, 0), (512, 777, 512, 4, 7, 0), (1024, 64, 1, 2, 8, 0),
        (128, 129, 128, 1, 9, 0), (2048, 3000, 41, 37, 10, 8),
        # one accumulation chunk of 9000 samples (listed 4096 at a time), a 32-cluster assignment window
        (256, 9000, 13, 30, 11, 0)]


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


def log(msg):
    print(msg, flush=True)


def nerr(a, b):
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def make_X(p, n, K, seed, ld_extra):
    rng = np.random.default_rng([p, n, seed])
    C = rng.standard_normal((K, p)) * 2.0
    lab = rng.integers(0, K, size=n)
    X = (C[lab] + rng.standard_normal((n, p))).astype(np.float32)
    Xl = np.zeros((n, p + ld_extra), dtype=np.float32)
    Xl[:, :p] = X
    return X, Xl


def oracle_seed_centers(vals, idx, p, K):
    C = np.zeros((K, p))
    for k in range(min(K, len(vals))):
        C[k, idx[k].astype(np.int64)] = vals[k]
    return C


@pytest.fixture(scope="module")
def data():
    out = []
    for (p, n, m, K, seed, ldx) in SETS:
        X, Xl = make_X(p, n, K, seed, ldx)
        vals, idx = ref.compress(X, seed, m) if n > 0 else (np.zeros((0, m)), np.zeros((0, m), np.uint16))
        out.append(dict(p=p, n=n, m=m, K=K, seed=seed, X=X, Xl=Xl, ovals=vals, oidx=idx))
    return out


def build(data, T):
    sets = []
    for d in data:
        Xt = torch.from_numpy(d["Xl"]).cuda()[:, :d["p"]] if d["n"] > 0 else torch.empty(
            (0, d["p"]), dtype=torch.float32, device="cuda")
        sets.append(dict(X=Xt, m=d["m"], K=d["K"], seed=d["seed"]))
    return Batch(sets, T=T)


def oracle_rounds(d, T):
    C = oracle_seed_centers(d["ovals"], d["oidx"], d["p"], d["K"])
    objs, assign = [], None
    for _ in range(T):
        if d["n"] == 0:
            objs.append(0.0)
            continue
        C, assign, obj, _ = ref.kmeans_step(d["p"], d["ovals"], d["oidx"], C)
        objs.append(obj)
    return C, assign, np.array(objs)


def test_batch_compress_matches_oracle(data):
    b = build(data, T=0)
    log(f"batch info {b.info()}")
    b.compress()
    torch.cuda.synchronize()
    for d, s in zip(data, b.sets):
        log(f"  set p={d['p']} n={d['n']} m={d['m']}")
        if d["n"] == 0:
            continue
        idx = s["idx"].cpu().numpy().view(np.uint16)
        assert np.array_equal(idx, d["oidx"])
        assert nerr(s["vals"].cpu().numpy(), d["ovals"]) < 1e-6


def test_batch_compress_equals_single_plan_calls(data):
    b = build(data, T=0)
    b.compress()
    for d, s in zip(data, b.sets):
        if d["n"] == 0:
            continue
        plan = pds.Plan(d["p"], d["m"], seed=d["seed"], prec=pds.PDS_F32)
        v1, i1 = pds.compress(plan, s["X"])
        torch.cuda.synchronize()
        assert torch.equal(i1, s["idx"])
        if d["p"] >= 256:  # the same transform code: bit-identical values
            assert torch.equal(v1, s["vals"])


@pytest.mark.parametrize("T", [1, 2, 5])
def test_batch_kmeans_matches_oracle(data, T):
    b = build(data, T=T)
    b.compress()
    b.init_centers()
    torch.cuda.synchronize()
    for d, s in zip(data, b.sets):
        C0 = oracle_seed_centers(d["ovals"], d["oidx"], d["p"], d["K"])
        assert nerr(s["centers"].cpu().numpy(), C0) < 1e-6 or d["n"] == 0
    b.kmeans()
    torch.cuda.synchronize()
    for d, s in zip(data, b.sets):
        C, assign, objs = oracle_rounds(d, T)
        log(f"  T={T} set p={d['p']} n={d['n']} K={d['K']}: objective gpu "
            f"{s['objective'].cpu().numpy()[:T]} oracle {objs}")
        assert nerr(s["centers"].cpu().numpy(), C) < 1e-5
        if d["n"] > 0:
            assert np.array_equal(s["assign"].cpu().numpy(), assign)
            o = s["objective"].cpu().numpy()[:T]
            assert np.allclose(o, objs, rtol=1e-5, atol=1e-9)
            assert np.all(np.diff(o) <= 1e-6 * o[0])  # J' is non-increasing


def test_batch_graph_replays(data):
    T = 3
    b = build(data, T=T)
    b.compress()
    ref_out = [oracle_rounds(d, T) for d in data]
    results = []
    for rep in range(3):
        b.init_centers()
        b.kmeans()
        torch.cuda.synchronize()
        # eager work between replays: a single-set call on the same stream
        d0, s0 = data[3], b.sets[3]
        plan = pds.Plan(d0["p"], d0["m"], seed=d0["seed"])
        pds.kmeans_step(plan, s0["vals"], s0["idx"], s0["centers"].clone())
        torch.cuda.synchronize()
        results.append([(s["centers"].cpu().numpy().copy(), s["assign"].cpu().numpy().copy()) for s in b.sets])
    for rep in range(3):
        for d, (C, a), (Co, ao, _) in zip(data, results[rep], ref_out):
            assert nerr(C, Co) < 1e-5
            if d["n"] > 0:
                assert np.array_equal(a, ao)
        for (C, a), (C0, a0) in zip(results[rep], results[0]):
            assert np.array_equal(a, a0)
            assert nerr(C, C0) < 1e-6


def test_batch_autotune_keeps_results(data):
    T = 2
    b = build(data, T=T)
    b.compress()
    b.init_centers()
    before = [s["idx"].clone() for s in b.sets]
    b.autotune()
    info = b.info()
    log(f"autotuned: {info}")
    assert int(info["spw"]) in (16, 32, 64)
    b.compress()
    b.init_centers()
    b.kmeans()
    torch.cuda.synchronize()
    for d, s, i0 in zip(data, b.sets, before):
        assert torch.equal(s["idx"], i0)
        C, assign, _ = oracle_rounds(d, T)
        assert nerr(s["centers"].cpu().numpy(), C) < 1e-5
        if d["n"] > 0:
            assert np.array_equal(s["assign"].cpu().numpy(), assign)


@pytest.fixture(scope="module")
def drawn():
    """24 sets drawn (seeded) from the benched 256-set workload, each with its own
    p, m, K and seed and that workload's data recipe, rows capped at 2000-2499
    (ragged) so the oracle stays fast; 12 further sets keep their full n (below
    12000 rows) so accumulation chunks and long work-queue items are exercised."""
    prm = synth.batch_params("batch256_f32")
    rng = np.random.default_rng(20261203)
    small = [int(i) for i in rng.choice(len(prm), 24, replace=False)]
    full = [i for i in range(len(prm)) if prm[i]["n"] <= 12000 and i not in small][:12]
    out = []
    for j, i in enumerate(small + full):
        pr = prm[i]
        n = pr["n"] if i in full else min(pr["n"], 2000 + (i * 37) % 500)
        X = synth.batch_set_torch("batch256_f32", i, pr, n=n)
        Xh = X.cpu().numpy()
        v, ix = ref.compress(Xh, pr["seed"], pr["m"])
        out.append(dict(p=pr["p"], n=n, m=pr["m"], K=pr["K"], seed=pr["seed"], X=X, ovals=v, oidx=ix, set=i))
    torch.cuda.synchronize()
    return out


def test_batch_draw_of_benched_workload(drawn):
    """The batched form on sets drawn from the benched workload: kept indices
    bit-exact and values 1e-6 for every set; after T = 3 rounds (GPU seeding
    rule on both sides) centers and objectives within 1e-5, and every
    assignment equal to the oracle's except where the oracle's own margin is
    below the FP32 noise of a distance (the GPU clusters its FP32 values, the
    oracle its FP64 ones)."""
    T = 3
    b = Batch([dict(X=d["X"], m=d["m"], K=d["K"], seed=d["seed"]) for d in drawn], T=T)
    b.compress()
    b.init_centers()
    b.kmeans()
    torch.cuda.synchronize()
    for d, s in zip(drawn, b.sets):
        log(f"  set {d['set']}: p={d['p']} n={d['n']} m={d['m']} K={d['K']}")
        assert np.array_equal(s["idx"].cpu().numpy().view(np.uint16), d["oidx"])
        assert nerr(s["vals"].cpu().numpy(), d["ovals"]) < 1e-6
        C = oracle_seed_centers(d["ovals"], d["oidx"], d["p"], d["K"])
        objs = []
        for _ in range(T):
            C, a_o, J_o, margin = ref.kmeans_step(d["p"], d["ovals"], d["oidx"], C)
            objs.append(J_o)
        assert nerr(s["centers"].cpu().numpy(), C) < 1e-5
        bad = np.nonzero(s["assign"].cpu().numpy() != a_o)[0]
        assert np.all(margin[bad] <= 1e-4 * (J_o / d["n"])), (d["set"], bad[:5], margin[bad][:5])
        assert np.allclose(s["objective"].cpu().numpy()[:T], objs, rtol=1e-5, atol=1e-9)


def _create_status(p, m, K, align_off=0, reserved=0):
    X = torch.zeros((10, p + 8), dtype=torch.float32, device="cuda")
    d = (_lib.PdsBatchDesc * 1)()
    c = torch.zeros((K, p), dtype=torch.float64, device="cuda")
    c2 = torch.zeros((K, p), dtype=torch.float64, device="cuda")
    v = torch.zeros((10, max(m, 1)), dtype=torch.float32, device="cuda")
    i = torch.zeros((10, max(m, 1)), dtype=torch.int16, device="cuda")
    a = torch.zeros(10, dtype=torch.int32, device="cuda")
    o = torch.zeros(4, dtype=torch.float64, device="cuda")
    d[0].X, d[0].n, d[0].ldx, d[0].p, d[0].m, d[0].K = X.data_ptr() + 4 * align_off, 10, p + 8, p, m, K
    d[0].reserved, d[0].seed = reserved, 0
    d[0].vals, d[0].idx, d[0].centers, d[0].centers_alt = v.data_ptr(), i.data_ptr(), c.data_ptr(), c2.data_ptr()
    d[0].assign, d[0].objective = a.data_ptr(), o.data_ptr()
    h = ctypes.c_void_p()
    st = _lib.lib().pds_batch_create(ctypes.byref(h), d, 1, 2)
    if st == 0:
        _lib.lib().pds_batch_destroy(h)
    return st


def test_batch_argument_errors():
    assert _create_status(256, 26, 3) == 0
    assert _create_status(64, 6, 3) == _lib.PDS_E_UNSUPPORTED
    assert _create_status(4096, 6, 3) == _lib.PDS_E_UNSUPPORTED
    assert _create_status(256, 257, 3) == _lib.PDS_E_M
    assert _create_status(256, 26, 0) == _lib.PDS_E_ARG
    assert _create_status(256, 26, 3, align_off=1) == _lib.PDS_E_ARG
    assert _create_status(128, 26, 3, align_off=1) == 0  # p = 128 reads scalars: no alignment needed
    assert _create_status(256, 26, 3, reserved=1) == _lib.PDS_E_ARG
