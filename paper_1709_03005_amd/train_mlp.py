"""Train the learned Davidson preconditioner on Hamiltonians built by this
library (seeded training instances, D ~ U[2000, 20000]).

For every training instance:
  1. build the contracted matrix and solve for the lowest k pairs tightly
     (Jacobi step) -> reference eigenvectors x*;
  2. run the solver again stopped after a few iteration counts; each stopped
     run gives Ritz pairs (theta, x) and residuals r (returned by the library);
  3. for each unconverged pair, the target correction is the error of the Ritz
     vector, e = x*/(x . x*) - x, the Jacobi step tj = r / (theta - H_ii)
     (denominator floored at 1e-8), and the row features come from
     cch_mlp_features(theta); each state's rows (tj and e together) are scaled
     by 1 / rms(e) over its sampled rows, so that every state weighs the same
     and the FP32 loss stays O(1).
Training: Adam on the device (cch_mlp_train_step), minibatches of rows.
Afterwards a few held-out instances are solved with the Jacobi and the
learned corrections and the iteration counts are printed side by side.

Usage: python -m paper_1709_03005_amd.train_mlp --instances 200 --out weights.npy
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def collect_rows(cc, ctx, k=10, stops=(1, 2, 3, 5, 8, 12), rows_per_state=4096, rng=None):
    """(X, tj, e, w) rows from stopped Davidson runs on a built context."""
    rng = rng or np.random.default_rng(0)
    ev, xs, info, rc = ctx.davidson(k, tol=1e-10, max_iter=400)
    diag = ctx.get_diagonal()
    out = []
    for j in stops:
        th, vr, _, _ = ctx.davidson(k, tol=1e-10, max_iter=j, residuals=True)
        V, R = vr[:k], vr[k:]
        for e in range(k):
            x, r, t = V[e], R[e], th[e]
            rn = np.linalg.norm(r)
            if not np.isfinite(rn) or rn < 1e-9:
                continue
            ov = float(x @ xs[e])
            if abs(ov) < 0.2:
                continue
            target = xs[e] / ov - x
            tn = float(target @ target)
            if not np.isfinite(tn) or tn == 0.0:
                continue
            den = t - diag
            den = np.where(np.abs(den) < 1e-8, np.where(den < 0, -1e-8, 1e-8), den)
            tj = r / den
            F = ctx.mlp_features(float(t))
            sel = rng.choice(len(x), size=min(rows_per_state, len(x)), replace=False)
            rms = float(np.sqrt(np.mean(target[sel] ** 2)))
            if not np.isfinite(rms) or rms == 0.0:
                continue
            out.append((F[sel], tj[sel] / rms, target[sel] / rms, np.ones(len(sel))))
    if not out:
        return None
    X = np.concatenate([o[0] for o in out]).astype(np.float32)
    tj = np.concatenate([o[1] for o in out]).astype(np.float32)
    e = np.concatenate([o[2] for o in out]).astype(np.float32)
    w = np.concatenate([o[3] for o in out]).astype(np.float32)
    return X, tj, e, w


def train(instances=200, out=None, seed=0, epochs=20, batch=65536, lr=1e-3, max_seconds=None, n_eval=4,
          log=print):
    import torch

    import paper_1709_03005_amd as cc
    import synth
    torch.cuda.init()
    t0 = time.time()
    net = cc.Mlp(seed=seed)
    data = []
    rng = np.random.default_rng(seed)
    used = 0
    for i in range(instances):
        if max_seconds and time.time() - t0 > 0.6 * max_seconds:
            break
        inst = synth.learned_train(i)
        with cc.from_instance(inst) as ctx:
            ctx.build()
            rows = collect_rows(cc, ctx, rng=rng)
        if rows is not None:
            data.append(rows)
            used += 1
        log(f"[train] instance {i}: D={inst.dim()} rows={0 if rows is None else len(rows[0])} "
            f"t={time.time() - t0:.0f}s")
    X = np.concatenate([d[0] for d in data])
    tj = np.concatenate([d[1] for d in data])
    e = np.concatenate([d[2] for d in data])
    w = np.concatenate([d[3] for d in data])
    dev = torch.device("cuda")
    Xd, tjd, ed, wd = (torch.from_numpy(a).to(dev) for a in (X, tj, e, w))
    n = len(X)
    losses = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(dev)
        tot = 0.0
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            tot += net.train_step(Xd[idx].contiguous(), tjd[idx].contiguous(), ed[idx].contiguous(),
                                  wd[idx].contiguous(), lr=lr)
        losses.append(tot / n)
        log(f"[train] epoch {ep}: mean loss {losses[-1]:.5f} t={time.time() - t0:.0f}s")
        if max_seconds and time.time() - t0 > max_seconds:
            break
    wts = net.weights()
    if out:
        np.save(out, wts)
    held = evaluate(cc, synth, net, n_eval=n_eval, log=log) if n_eval else []
    net.close()
    return wts, {"instances": used, "rows": n, "losses": losses, "seconds": time.time() - t0,
                 "held_out": held}


def evaluate(cc, synth, net, n_eval=4, k=10, tol=1e-8, log=print):
    """Jacobi vs learned corrections on held-out instances (seeds disjoint
    from the training draws)."""
    res = []
    for i in range(n_eval):
        inst = synth.learned_train(1000 + i)
        with cc.from_instance(inst) as ctx:
            ctx.build()
            ev_j, _, inf_j, _ = ctx.davidson(k, tol=tol, max_iter=400, want_vectors=False)
            ctx.set_mlp(net)
            ev_m, _, inf_m, _ = ctx.davidson(k, tol=tol, max_iter=400, want_vectors=False,
                                             precond=cc.CCH_PRECOND_MLP)
            ctx.set_mlp(None)
        r = dict(D=inst.dim(), jacobi_iter=inf_j.iterations, mlp_iter=inf_m.iterations,
                 jacobi_ms=1e3 * inf_j.seconds, mlp_ms=1e3 * inf_m.seconds,
                 fallbacks=inf_m.fallbacks, max_dev=float(np.max(np.abs(ev_j - ev_m))))
        log(f"[eval] {r}")
        res.append(r)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--instances", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "mlp_weights.npy"))
    ap.add_argument("--max-seconds", type=float, default=None)
    args = ap.parse_args()
    _, info = train(args.instances, args.out, epochs=args.epochs, max_seconds=args.max_seconds,
                    log=lambda s: print(s, flush=True))
    print(info)


if __name__ == "__main__":
    main()
