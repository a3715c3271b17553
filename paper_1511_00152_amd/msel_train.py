"""Trains and evaluates the learned m-selector on synthetic p = 1024, n = 8192
blocks (the ``msel`` generator of ``synth``), on the GPU.

    python -m paper_1511_00152_amd.msel_train --train 100000 --heldout 10000 \\
        --out-dir DIR [--install]

Steps: (1) features and labels of the training blocks (stream 1); (2) FP32
training of the network; (3) on held-out blocks (stream 2): the selector's m
(BF16 inference), the realized relative Frobenius error of the covariance
estimator at that m, at the label m and at the fixed comparison m = 0.2 p.
The selector's fallback (for blocks whose features or output are not finite)
is then set to the smallest single fixed m that meets the target on as many
held-out blocks as the selector does: a conservative m measured on data the
network did not see.
Writes DIR/msel_eval.json (and the weights when --install is given, into the
package).  Progress goes to stdout as the work proceeds.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=100000)
    ap.add_argument("--heldout", type=int, default=10000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch-blocks", type=int, default=64, help="blocks per batched basis draw")
    ap.add_argument("--out-dir", default="msel_out")
    ap.add_argument("--install", action="store_true", help="write the trained weights into the package")
    ap.add_argument("--save-data", default=None, help="write the training features and labels (npz)")
    ap.add_argument("--load-data", default=None, help="train on features and labels from an npz instead")
    args = ap.parse_args(argv)

    import torch

    import synth
    import paper_1511_00152_amd as pds
    from paper_1511_00152_amd import msel

    if not torch.cuda.is_available():
        raise SystemExit("a GPU is required")
    os.makedirs(args.out_dir, exist_ok=True)
    cfg = synth.MSEL
    p, n, t, nsub = cfg["p"], cfg["n"], cfg["target"], cfg["nsub"]
    dev = "cuda"
    ctx = msel.MselContext(p=p, n=n, seed=0, device=dev)

    def log(msg):
        print(msg, flush=True)

    def featurize(stream, count, keep=None):
        feats = torch.empty((count, msel.N_FEAT), dtype=torch.float32, device=dev)
        labels = torch.empty(count, dtype=torch.int32, device=dev)
        t0 = time.time()
        done = 0
        for b0 in range(0, count, args.batch_blocks):
            c = min(args.batch_blocks, count - b0)
            for k, (X, prm) in enumerate(synth.msel_blocks_torch(stream, b0, c, device=dev)):
                i = b0 + k
                ctx.features(X, nsub=nsub, target=t, out=feats[i])
                ctx.label(X, target=t, m_out=labels[i:i + 1])
                if keep is not None:
                    keep(i, X, prm)
            done += c
            if done % 2048 < args.batch_blocks or done == count:
                torch.cuda.synchronize()
                el = time.time() - t0
                log(f"stream {stream}: {done}/{count} blocks, {el:.1f} s, {1e3 * el / done:.2f} ms/block")
        torch.cuda.synchronize()
        return feats, labels, time.time() - t0

    # (1) training set
    if args.load_data:
        z = np.load(args.load_data, allow_pickle=False)
        ftr = torch.as_tensor(z["feats"], device=dev).contiguous()
        ltr = torch.as_tensor(z["labels"], device=dev).contiguous()
        t_gen = float(z["seconds"])
        log(f"loaded {ftr.shape[0]} training blocks from {args.load_data}")
    else:
        log(f"generating {args.train} training blocks (p={p}, n={n}, target {t})")
        ftr, ltr, t_gen = featurize(1, args.train)
        if args.save_data:
            np.savez(args.save_data, feats=ftr.cpu().numpy(), labels=ltr.cpu().numpy(), seconds=np.float64(t_gen))
    ytr = torch.log(ltr.float() / p)
    bad = ~torch.isfinite(ftr).all(1)
    if bool(bad.any()):
        log(f"dropping {int(bad.sum())} blocks with non-finite features")
        ftr, ytr = ftr[~bad].contiguous(), ytr[~bad].contiguous()

    # (2) training
    t0 = time.time()
    sel = msel.MSelector.fit(ftr, ytr.contiguous(), epochs=args.epochs, log=log, target=t, nsub=nsub, p=p)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    log(f"training: {t_train:.1f} s")

    # (3) held-out evaluation
    m_fix = msel.m_from_gamma(cfg["gamma_baseline"], p)
    plans = {}

    def plan_for(m):
        if m not in plans:
            plans[m] = pds.Plan(p, m, ctx.seed, pds.PDS_F32)  # same D as the exact covariance
        return plans[m]

    cov_ws = {"t": None}
    C_ex = torch.empty((p, p), dtype=torch.float64, device=dev)
    C_hat = torch.empty((p, p), dtype=torch.float64, device=dev)
    acc = torch.empty((p, p), dtype=torch.float64, device=dev)
    vals = torch.empty(n * p, dtype=torch.float32, device=dev)
    idx = torch.empty(n * p, dtype=torch.int16, device=dev)
    fws = torch.empty(4096, dtype=torch.uint8, device=dev)
    rows = []

    def realized(X, m, i):
        pl = plan_for(m)
        need = pl.workspace_size(pds.PDS_OP_COVARIANCE, n)
        if cov_ws["t"] is None or cov_ws["t"].numel() < need:
            cov_ws["t"] = torch.empty(need, dtype=torch.uint8, device=dev)
        v, ix = vals[:n * m].view(n, m), idx[:n * m].view(n, m)
        pds.compress(pl, X, i0=i * n, vals=v, idx=ix)
        acc.zero_()
        pds.covariance(pl, v, ix, acc=acc, ws=cov_ws["t"], C=C_hat)
        return msel.frob_diff(C_hat, C_ex, ws=fws)

    t0 = time.time()
    ho_feats, ho_labels = [], []
    for b0 in range(0, args.heldout, args.batch_blocks):
        c = min(args.batch_blocks, args.heldout - b0)
        for k, (X, prm) in enumerate(synth.msel_blocks_torch(2, b0, c, device=dev)):
            i = b0 + k
            f = ctx.features(X, nsub=nsub, target=t)
            lab = ctx.label(X, target=t, C_out=C_ex)
            g = sel.predict_gamma(f)
            m_sel = msel.m_from_gamma(float(g[0]), p)
            m_lab = int(lab[0])
            errs = {}
            for name, m in (("selector", m_sel), ("label", m_lab), ("fixed", m_fix)):
                if m >= p:
                    errs[name] = 0.0
                    continue
                d = realized(X, m, i)
                errs[name] = math.sqrt(float(d[0]) / float(d[1]))
            ho_feats.append(f)
            rows.append(dict(block=i, r=prm["r"], alpha=prm["alpha"], amp=prm["amp"], m_sel=m_sel, m_label=m_lab,
                             err_sel=errs["selector"], err_label=errs["label"], err_fixed=errs["fixed"]))
        done = b0 + c
        if done % 1024 < args.batch_blocks or done == args.heldout:
            el = time.time() - t0
            log(f"held-out: {done}/{args.heldout} blocks, {el:.1f} s")
    t_eval = time.time() - t0

    m_sel = np.array([r["m_sel"] for r in rows], dtype=np.float64)
    m_lab = np.array([r["m_label"] for r in rows], dtype=np.float64)
    e_sel = np.array([r["err_sel"] for r in rows])
    e_lab = np.array([r["err_label"] for r in rows])
    e_fix = np.array([r["err_fixed"] for r in rows])
    ok_sel = float((e_sel <= t).mean())
    # smallest single fixed m that would have met the label on the same share of blocks
    m_equal = float(np.quantile(m_lab, ok_sel, method="higher")) if len(m_lab) else float("nan")
    summary = dict(
        p=p, n=n, target=t, nsub=nsub, train_blocks=int(ftr.shape[0]), heldout_blocks=len(rows),
        time_s=dict(train_data=round(t_gen, 1), training=round(t_train, 1), heldout_eval=round(t_eval, 1)),
        ms_per_train_block=round(1e3 * t_gen / max(int(ltr.shape[0]), 1), 3),
        selector=dict(success=ok_sel, mean_gamma=float(m_sel.mean() / p), median_gamma=float(np.median(m_sel) / p)),
        label=dict(success=float((e_lab <= t).mean()), mean_gamma=float(m_lab.mean() / p)),
        fixed_baseline=dict(m=m_fix, success=float((e_fix <= t).mean()), mean_gamma=m_fix / p),
        fixed_m_for_same_success=dict(m=m_equal, gamma=m_equal / p),
        log_ratio_sel_over_label=dict(mean=float(np.log(m_sel / m_lab).mean()),
                                      mae=float(np.abs(np.log(m_sel / m_lab)).mean())),
        realized_err=dict(sel_median=float(np.median(e_sel)), label_median=float(np.median(e_lab))),
    )
    sel.meta.update(summary)
    sel.gamma_fallback = m_equal / p
    with open(os.path.join(args.out_dir, "msel_eval.json"), "w") as f:
        json.dump(summary, f, indent=1, sort_keys=True)
    with open(os.path.join(args.out_dir, "msel_heldout_rows.json"), "w") as f:
        json.dump(rows, f)
    sel.save(os.path.join(args.out_dir, "msel_p1024.npz"), os.path.join(args.out_dir, "msel_p1024.json"))
    if args.install:
        sel.save()
    log(json.dumps(summary))
    return 0


if __name__ == "__main__":
    sys.exit(main())
