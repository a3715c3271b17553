"""Pins of the m-selector oracle (CPU, no GPU): the expected-error formula by
enumerating every sampling outcome, Monte Carlo agreement with the C oracle's
estimator, the feature statistics by brute force and library routines, and
the network's gradient and optimizer by finite differences and torch."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import msel as om
from oracle import oracle_def, ref


def _exact_mean_sq_error(Y, m):
    """Average of ||C_n - C_emp||_F^2 over every combination of kept sets
    (one m-subset per sample), with the literal estimator (Sec. V)."""
    n, p = Y.shape
    Yc = Y.T  # p x n, one sample per column as the paper writes it
    Ce = oracle_def.cov_emp(Yc)
    subsets = list(itertools.combinations(range(p), m))
    tot = 0.0
    cnt = 0
    for combo in itertools.product(subsets, repeat=n):
        idx = [np.array(s) for s in combo]
        Cn = oracle_def.cov_n(Yc, idx, m)
        tot += float(((Cn - Ce) ** 2).sum())
        cnt += 1
    return tot / cnt


@pytest.mark.parametrize("p,m,n", [(6, 2, 1), (6, 3, 1), (6, 4, 2), (6, 3, 2), (4, 2, 2), (5, 5, 1)])
def test_expected_error_equals_enumeration(p, m, n):
    Y = np.random.default_rng([p, m, n]).standard_normal((n, p))
    e2 = om.expected_e2(Y, m)
    Ce = Y.T @ Y / n
    exact = _exact_mean_sq_error(Y, m) / float((Ce * Ce).sum())
    assert e2 == pytest.approx(exact, rel=1e-12, abs=1e-15)


def test_expected_error_matches_monte_carlo_of_the_c_oracle():
    # realized errors of the C oracle's compress + covariance over many seeds
    p, n, m = 64, 128, 16
    X = np.random.default_rng(5).standard_normal((n, p))
    X[:, 3] *= 6.0
    errs = []
    for seed in range(150):
        D = ref.signs(seed, p)
        Y = om.transform(X, D)
        vals, idx = ref.compress(X, seed, m)
        C = ref.covariance(p, vals, idx)
        Ce = Y.T @ Y / n
        errs.append(float(((C - Ce) ** 2).sum()) / float((Ce * Ce).sum()) / om.expected_e2(Y, m))
    # each ratio has mean 1 (the expectation is over the sampling, D fixed per seed)
    r = np.array(errs)
    assert abs(r.mean() - 1.0) < 4.0 * r.std() / math.sqrt(len(r)) + 0.02


def test_label_is_the_smallest_m_meeting_the_target():
    X, _ = synth.msel_block_numpy(0, 1, p=64, n=256)
    Y = om.transform(X, ref.signs(0, 64))
    t = 0.3
    m = om.label_m(Y, t)
    e = [om.expected_e2(Y, k) for k in range(2, 65)]
    assert all(e[i] >= e[i + 1] for i in range(len(e) - 1))
    assert e[m - 2] <= t * t and (m == 2 or e[m - 3] > t * t)
    assert om.expected_e2(Y, 64) == 0.0


def test_label_of_zero_block_and_tight_target():
    assert om.label_m(np.zeros((8, 16)), 0.1) == 2
    Y = np.random.default_rng(2).standard_normal((4, 16))
    assert om.label_m(Y, 1e-9) == 16


@pytest.mark.parametrize("s", [2, 3, 10, 37, 512, 1000])
def test_quantile_rule_is_numpy_lower(s):
    v = np.random.default_rng(s).standard_normal(s)
    for q in om.QUANT_PER_MILLE:
        assert om.quantile_lower(v, q) == np.quantile(v, q / 1000.0, method="lower")


def test_pair_statistic_brute_force_and_plugin_label():
    p, s = 32, 40
    X = np.random.default_rng(9).standard_normal((s, p)) * np.linspace(0.5, 3.0, p)
    D = ref.signs(0, p)
    Y = om.transform(X, D)
    f = om.features(X, D, s, 0.2)
    pair = sum(float(Y[i] @ Y[k]) ** 2 for i in range(s) for k in range(s) if i != k) / (s * (s - 1))
    mean_y = (Y * Y).sum(1).mean()
    assert f[27] == pytest.approx(math.log(pair / mean_y ** 2), rel=1e-12)
    # with the whole block as the subset the plug-in moments are exact, so
    # feature 31 is the label itself
    assert f[31] == pytest.approx(math.log(om.label_m(Y, 0.2) / p), abs=1e-15)


def test_coherence_features_of_canonical_rows():
    # a row c e_j has raw coherence p and, after H D, is perfectly flat
    p, s = 64, 8
    X = np.zeros((s, p))
    for i in range(s):
        X[i, (5 * i) % p] = 1.0 + i
    f = om.features(X, ref.signs(3, p), s, 0.1)
    assert np.allclose(f[9:17], math.log(p), atol=1e-12)
    assert np.allclose(f[17:25], 0.0, atol=1e-12)
    assert f[25] == pytest.approx(0.0, abs=1e-12)  # flat: p sum y^4 / ||y||^4 = 1
    assert f[26] == pytest.approx(math.log(p), abs=1e-12)


def _params(seed):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal(om.N_PARAMS) * 0.3
    return P


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(1)
    B = 12
    F = rng.standard_normal((B, 32))
    mu, sd = rng.standard_normal(32) * 0.1, 1.0 + rng.random(32)
    tgt = rng.standard_normal(B)
    P = _params(2)
    g, _ = om.mlp_grad(P, F, mu, sd, tgt, 0.8)
    h = 1e-6
    for q in list(range(0, 2048, 97)) + list(range(2048, 6337, 113)) + [6336, 6335, 2100, 6250]:
        Pp, Pm = P.copy(), P.copy()
        Pp[q] += h
        Pm[q] -= h
        lp = om.expectile_loss(om.mlp_forward(Pp, F, mu, sd)[0], tgt, 0.8)
        lm = om.expectile_loss(om.mlp_forward(Pm, F, mu, sd)[0], tgt, 0.8)
        assert g[q] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-8), q


def test_mlp_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    B = 33
    F = rng.standard_normal((B, 32))
    mu, sd = rng.standard_normal(32) * 0.1, 1.0 + rng.random(32)
    tgt = rng.standard_normal(B)
    P = _params(4)
    tau = 0.9
    g, loss = om.mlp_grad(P, F, mu, sd, tgt, tau)
    Pt = torch.tensor(P, dtype=torch.float64, requires_grad=True)
    W1 = Pt[0:2048].view(64, 32)
    b1 = Pt[2048:2112]
    W2 = Pt[2112:6208].view(64, 64)
    b2 = Pt[6208:6272]
    w3 = Pt[6272:6336]
    b3 = Pt[6336]
    xn = (torch.tensor(F) - torch.tensor(mu)) / torch.tensor(sd)
    y = torch.relu(torch.relu(xn @ W1.T + b1) @ W2.T + b2) @ w3 + b3
    r = torch.tensor(tgt) - y
    w = torch.where(r < 0, torch.tensor(1 - tau, dtype=torch.float64), torch.tensor(tau, dtype=torch.float64))
    L = (w * r * r).mean()
    L.backward()
    assert loss == pytest.approx(float(L.detach()), rel=1e-13)
    np.testing.assert_allclose(g, Pt.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_expectile_half_is_half_mse():
    rng = np.random.default_rng(0)
    a, b = rng.standard_normal(50), rng.standard_normal(50)
    assert om.expectile_loss(a, b, 0.5) == pytest.approx(0.5 * float(((a - b) ** 2).mean()), rel=1e-14)


def test_adam_matches_torch_optim():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    P = rng.standard_normal(50)
    m1 = np.zeros(50)
    m2 = np.zeros(50)
    x = torch.tensor(P.copy(), requires_grad=True)
    opt = torch.optim.Adam([x], lr=0.01, betas=(0.9, 0.99), eps=1e-7)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        P, m1, m2 = om.adam_step(P, g, m1, m2, step, 0.01, 0.9, 0.99, 1e-7)
        opt.zero_grad()
        x.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(P, x.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    v = np.concatenate([rng.standard_normal(10000).astype(np.float32) * 10,
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, 1e-40], np.float32)])
    ours = om.bf16_round(v)
    theirs = torch.tensor(v).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours.view(np.uint32), theirs.view(np.uint32))
