"""Learned m-selector: chooses how many coordinates m to keep for a data block
so that the covariance estimator (Sec. V) meets a relative Frobenius error
target, from cheap statistics of the block's first rows.

Not part of the paper's method.  The training label of a block is the
smallest m whose expected squared relative error, over the method's own
sampling (inclusion probabilities of App. B), is at most target^2
(``pds_msel_label``).  A 32-64-64-1 network (FP32 training with an expectile
loss that penalizes choosing m too small, BF16 inference) maps the 32
features of ``pds_msel_features`` to log(m/p).

    ctx = MselContext(p=1024, n=8192)          # exact-transform plan + workspace
    sel = MSelector.load()                     # the shipped weights for p = 1024 blocks
    m = sel.choose_m(ctx, X)                   # X: n x p float32 on the GPU

Every numerical step runs in libpds kernels; this module only marshals
arguments (torch tensors supply device memory and the stream).
"""
import ctypes
import json
import math
import os

import numpy as np

from . import Plan, _ptr, _stream
from ._lib import PDS_F32, PDS_FROB_WS_BYTES, check, lib

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "msel_p1024.npz")
WEIGHTS_META = os.path.join(HERE, "msel_p1024.json")
N_FEAT = 32


def _torch():
    import torch

    return torch


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------
def row_moments(X, out=None):
    """(sum x^2, sum x^4, max x^2) per row of a float32 matrix, FP64 (n x 3)."""
    torch = _torch()
    n, p = X.shape
    if X.dtype != torch.float32 or X.stride(1) != 1:
        raise TypeError("X must be float32 with contiguous rows")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device=X.device)
    check(lib().pds_row_moments(_ptr(X), n, p, X.stride(0), _ptr(out), _stream()), "pds_row_moments")
    return out


def frob_diff(A, B, ws=None, out=None):
    """Device tensor (2,) FP64: (||A - B||_F^2, ||B||_F^2)."""
    torch = _torch()
    if A.shape != B.shape or A.dtype != torch.float64 or B.dtype != torch.float64:
        raise TypeError("A and B must be FP64 tensors of one shape")
    if ws is None:
        ws = torch.empty(PDS_FROB_WS_BYTES, dtype=torch.uint8, device=A.device)
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=A.device)
    check(lib().pds_frob_diff(_ptr(A.contiguous()), _ptr(B.contiguous()), A.numel(), _ptr(out), _ptr(ws), ws.numel(),
                              _stream()), "pds_frob_diff")
    return out


class MselContext:
    """The m = p plan (its compression is the exact transform y = H D x) and a
    workspace sized for blocks of up to n rows."""

    def __init__(self, p=1024, n=8192, seed=0, device="cuda"):
        torch = _torch()
        self.p, self.n, self.seed = int(p), int(n), int(seed)
        self.plan = Plan(self.p, self.p, self.seed, PDS_F32)
        b = ctypes.c_size_t(0)
        check(lib().pds_msel_workspace_size(self.plan.handle, self.n, ctypes.byref(b)), "pds_msel_workspace_size")
        self.ws = torch.empty(int(b.value), dtype=torch.uint8, device=device)
        self.device = device

    def _check_X(self, X):
        torch = _torch()
        if X.dtype != torch.float32 or X.stride(1) != 1 or X.shape[1] != self.p:
            raise TypeError(f"X must be float32, n x {self.p}, contiguous rows")
        if X.shape[0] > self.n:
            raise ValueError(f"block has {X.shape[0]} rows; the context was sized for {self.n}")

    def label(self, X, target=0.1, m_out=None, C_out=None):
        """Device int32 (1,): the label m of block X; C_out (p x p FP64) receives C_emp if given."""
        torch = _torch()
        self._check_X(X)
        if m_out is None:
            m_out = torch.empty(1, dtype=torch.int32, device=X.device)
        check(lib().pds_msel_label(self.plan.handle, _ptr(X), X.shape[0], X.stride(0), float(target), _ptr(m_out),
                                   _ptr(C_out), _ptr(self.ws), self.ws.numel(), _stream()), "pds_msel_label")
        return m_out

    def features(self, X, nsub=512, target=0.1, out=None):
        """Device float32 (32,): the features of block X from its first nsub rows."""
        torch = _torch()
        self._check_X(X)
        if out is None:
            out = torch.empty(N_FEAT, dtype=torch.float32, device=X.device)
        check(lib().pds_msel_features(self.plan.handle, _ptr(X), X.shape[0], X.stride(0), int(nsub), float(target),
                                      _ptr(out), _ptr(self.ws), self.ws.numel(), _stream()), "pds_msel_features")
        return out


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def mlp_param_count():
    return int(lib().pds_mlp_param_count())


def mlp_forward(params, feats, mu, sd, acts=None, pred=None):
    torch = _torch()
    B = feats.shape[0]
    if acts is None:
        acts = torch.empty((B, 160), dtype=torch.float32, device=feats.device)
    if pred is None:
        pred = torch.empty(B, dtype=torch.float32, device=feats.device)
    check(lib().pds_mlp_forward(_ptr(params), _ptr(feats), _ptr(mu), _ptr(sd), B, _ptr(acts), _ptr(pred), _stream()),
          "pds_mlp_forward")
    return pred, acts


def mlp_backward(params, acts, pred, target, tau, ws=None, grad=None, loss=None):
    torch = _torch()
    B = pred.shape[0]
    dev = pred.device
    if ws is None:
        ws = torch.empty(B * 130, dtype=torch.float32, device=dev)
    if grad is None:
        grad = torch.empty(mlp_param_count(), dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
    check(lib().pds_mlp_backward(_ptr(params), _ptr(acts), _ptr(pred), _ptr(target), B, float(tau), _ptr(ws),
                                 ws.numel() * 4, _ptr(grad), _ptr(loss), _stream()), "pds_mlp_backward")
    return grad, loss


def mlp_adam(params, grad, m1, m2, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    check(lib().pds_mlp_adam(_ptr(params), _ptr(grad), _ptr(m1), _ptr(m2), int(step), float(lr), float(beta1),
                             float(beta2), float(eps), _stream()), "pds_mlp_adam")


def mlp_pack_bf16(params, out=None):
    torch = _torch()
    if out is None:
        out = torch.empty(mlp_param_count(), dtype=torch.int16, device=params.device)
    check(lib().pds_mlp_pack_bf16(_ptr(params), _ptr(out), _stream()), "pds_mlp_pack_bf16")
    return out


def msel_predict(params_bf16, feats, mu, sd, gamma_min, gamma_max, gamma_fallback, out=None):
    torch = _torch()
    B = feats.shape[0]
    if out is None:
        out = torch.empty(B, dtype=torch.float32, device=feats.device)
    check(lib().pds_msel_predict(_ptr(params_bf16), _ptr(feats), _ptr(mu), _ptr(sd), B, float(gamma_min),
                                 float(gamma_max), float(gamma_fallback), _ptr(out), _stream()), "pds_msel_predict")
    return out


def init_params(seed=0):
    """He-uniform weights, zero biases (numpy float32)."""
    rng = np.random.default_rng([seed, 0x3E1])
    P = np.zeros(mlp_param_count(), dtype=np.float32)
    P[0:2048] = rng.uniform(-1, 1, 2048) * math.sqrt(6.0 / 32)
    P[2112:6208] = rng.uniform(-1, 1, 4096) * math.sqrt(6.0 / 64)
    P[6272:6336] = rng.uniform(-1, 1, 64) * math.sqrt(6.0 / 64)
    return P


def m_from_gamma(gamma, p):
    """m = floor(gamma p + 1/2), clamped to [2, p]."""
    return max(2, min(p, int(math.floor(gamma * p + 0.5))))


class MSelector:
    """Trained selector: FP32 parameters, feature standardization, limits."""

    def __init__(self, params, mu, sd, target=0.1, tau=0.9, gamma_fallback=1.0, nsub=512, p=1024, meta=None,
                 device="cuda"):
        torch = _torch()
        self.params = torch.as_tensor(np.asarray(params, np.float32), device=device).contiguous()
        self.mu = torch.as_tensor(np.asarray(mu, np.float32), device=device).contiguous()
        self.sd = torch.as_tensor(np.asarray(sd, np.float32), device=device).contiguous()
        self.target, self.tau, self.gamma_fallback, self.nsub, self.p = target, tau, gamma_fallback, nsub, p
        self.meta = dict(meta or {})
        self._bf16 = None

    @staticmethod
    def standardization(feats):
        """Per-feature mean and scale of a training set (constant features get scale 1)."""
        torch = _torch()
        mu = feats.mean(0)
        sd = feats.std(0)
        sd = torch.where(sd > 1e-6, sd, torch.ones_like(sd))
        return mu, sd

    @classmethod
    def fit(cls, feats, labels_log_gamma, epochs=40, batch=512, lr=2e-3, tau=0.9, seed=0, log=None, **kw):
        """Train on device tensors feats (N x 32 float32), labels (N float32)."""
        torch = _torch()
        dev = feats.device
        mu, sd = cls.standardization(feats)
        sel = cls(init_params(seed), mu.cpu().numpy(), sd.cpu().numpy(), tau=tau, device=dev, **kw)
        P = sel.params
        m1 = torch.zeros_like(P)
        m2 = torch.zeros_like(P)
        N = feats.shape[0]
        g = torch.Generator(device=dev)
        g.manual_seed(seed)
        acts = torch.empty((batch, 160), dtype=torch.float32, device=dev)
        pred = torch.empty(batch, dtype=torch.float32, device=dev)
        ws = torch.empty(batch * 130, dtype=torch.float32, device=dev)
        grad = torch.empty_like(P)
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        step = 0
        nb = N // batch
        total = epochs * nb
        for ep in range(epochs):
            perm = torch.randperm(N, generator=g, device=dev)
            run = torch.zeros(1, dtype=torch.float32, device=dev)
            for k in range(nb):
                sel_idx = perm[k * batch:(k + 1) * batch]
                fb = feats[sel_idx].contiguous()
                tb = labels_log_gamma[sel_idx].contiguous()
                mlp_forward(P, fb, sel.mu, sel.sd, acts=acts, pred=pred)
                mlp_backward(P, acts, pred, tb, tau, ws=ws, grad=grad, loss=loss)
                step += 1
                # cosine decay of the step size to 5% of lr
                lr_t = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * step / total)))
                mlp_adam(P, grad, m1, m2, step, lr=lr_t)
                run += loss
            if log is not None:
                log(f"epoch {ep + 1}/{epochs} mean expectile loss {float(run) / max(nb, 1):.5f}")
        sel.meta.update(epochs=epochs, batch=batch, lr=lr, tau=tau, train_blocks=int(N))
        return sel

    def params_bf16(self):
        if self._bf16 is None:
            self._bf16 = mlp_pack_bf16(self.params)
        return self._bf16

    def predict_gamma(self, feats):
        """gamma for each row of feats (B x 32 device float32), BF16 inference."""
        f = feats.reshape(-1, N_FEAT).contiguous()
        return msel_predict(self.params_bf16(), f, self.mu, self.sd, 2.0 / self.p, 1.0, self.gamma_fallback)

    def choose_m(self, ctx, X):
        """m for block X (host int; synchronizes)."""
        g = self.predict_gamma(ctx.features(X, nsub=min(self.nsub, X.shape[0]), target=self.target))
        return m_from_gamma(float(g[0]), self.p)

    def save(self, path=WEIGHTS, meta_path=WEIGHTS_META):
        np.savez(path, params=self.params.cpu().numpy(), mu=self.mu.cpu().numpy(), sd=self.sd.cpu().numpy())
        meta = dict(self.meta, target=self.target, tau=self.tau, gamma_fallback=self.gamma_fallback, nsub=self.nsub,
                    p=self.p)
        with open(meta_path, "w") as f:
            json.dump(meta, f, indent=1, sort_keys=True)

    @classmethod
    def load(cls, path=WEIGHTS, meta_path=WEIGHTS_META, device="cuda"):
        z = np.load(path, allow_pickle=False)
        with open(meta_path) as f:
            meta = json.load(f)
        return cls(z["params"], z["mu"], z["sd"], target=meta["target"], tau=meta["tau"],
                   gamma_fallback=meta["gamma_fallback"], nsub=meta["nsub"], p=meta["p"], meta=meta, device=device)
