"""Learned warm start for the SSN solver: data generation, training and storage of the network.

The network (3 layers, width H) maps the size-independent per-filling-point features of ``kot_features`` to
t_i = gamma_i / lambda1.  Training data are duals of generated problems solved by the plain SSN solver on the
GPU; the forward/backward passes and Adam run in the library's kernels (``kot_mlp_loss_grad``,
``kot_mlp_adam``).  Feature standardization is folded into the first layer when the weights are saved, so
inference takes the raw features.

    python -m paper_2310_14087_amd.warmstart --problems 4096 --epochs 30 --out <file.npz>
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from pathlib import Path

import numpy as np

F_DEFAULT = 12
H_DEFAULT = 512
DEFAULT_WEIGHTS = Path(__file__).resolve().parent / "weights" / "warmstart_mix256.npz"


def _log(msg):
    print(f"[warmstart] {msg}", file=sys.stderr, flush=True)


def build_dataset(ctx, seeds, workload="mix256", l=None, n=None):
    """Solve each generated problem with plain SSN (cold start) and collect (features, gamma/lambda1)."""
    import torch
    from . import kotssn
    from .inputs import make_problem
    Xs, ys, info = [], [], []
    dev = torch.device("cuda:0")
    t_start = time.perf_counter()
    for cnt, s in enumerate(seeds):
        if cnt and cnt % 256 == 0:
            _log(f"dataset: {cnt} problems solved ({time.perf_counter() - t_start:.1f} s)")
        p = make_problem(workload, s, l=l, n=n)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        xs, yy, xf, yf = t(p.xs), t(p.ys), t(p.xf), t(p.yf)
        prm = kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol)
        gamma, _, r = ctx.solve(xs, yy, xf, yf, prm)
        info.append(dict(seed=s, status=r.status, iters=r.iters, ms=r.time_ms))
        if r.status != kotssn.KOT_OK:
            continue
        Q, z, R, wsum, q2 = ctx.setup(xs, yy, xf, yf, prm)
        X = ctx.features(Q, z, R, wsum, q2, prm)
        Xs.append(X.cpu().numpy())
        ys.append((gamma / p.lam1).float().cpu().numpy())
    return np.concatenate(Xs), np.concatenate(ys), info


def init_theta(F, H, seed=0):
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((F, H)) * np.sqrt(2.0 / F)
    W2 = rng.standard_normal((H, H)) * np.sqrt(2.0 / H)
    W3 = rng.standard_normal((H, 1)) * np.sqrt(1.0 / H)
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), np.zeros(1)]).astype(np.float32)


def standardize_stats(X):
    mu = X.astype(np.float64).mean(axis=0)
    sd = X.astype(np.float64).std(axis=0)
    sd[sd < 1e-12] = 1.0
    return mu, sd


def fold_standardization(theta, mu, sd, F, H):
    """Weights for raw x from weights trained on (x - mu)/sd: W1' = W1/sd, b1' = b1 - (mu/sd) W1."""
    th = theta.astype(np.float64).copy()
    W1 = th[:F * H].reshape(F, H)
    b1 = th[F * H:F * H + H]
    b1_new = b1 - (mu / sd) @ W1
    W1_new = W1 / sd[:, None]
    th[:F * H] = W1_new.ravel()
    th[F * H:F * H + H] = b1_new
    return th.astype(np.float32)


def fit(ctx, X, y, H=H_DEFAULT, epochs=30, batch=4096, lr=1e-3, seed=0, log_every=5):
    """Adam on the MSE of t = gamma/lambda1, all passes on the GPU.  Returns (folded theta, history)."""
    import torch
    F = X.shape[1]
    mu, sd = standardize_stats(X)
    dev = torch.device("cuda:0")
    Xg = torch.from_numpy(((X - mu) / sd).astype(np.float32)).to(dev)
    yg = torch.from_numpy(y.astype(np.float32)).to(dev)
    theta = torch.from_numpy(init_theta(F, H, seed)).to(dev)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.empty_like(theta)
    rng = np.random.default_rng(seed + 1)
    N = X.shape[0]
    step = 0
    hist = []
    for ep in range(epochs):
        lr_ep = lr * 0.5 * (1.0 + np.cos(np.pi * ep / epochs))   # cosine decay
        perm = torch.from_numpy(rng.permutation(N)).to(dev)
        tot, cnt = 0.0, 0
        for b0 in range(0, N - batch + 1 if N >= batch else 1, batch):
            idx = perm[b0:b0 + batch]
            xb = Xg[idx].contiguous()
            yb = yg[idx].contiguous()
            loss, _ = ctx.mlp_loss_grad(xb, yb, theta, H, grad)
            step += 1
            ctx.mlp_adam(theta, grad, m, v, step, lr=lr_ep)
            tot += loss * xb.shape[0]
            cnt += xb.shape[0]
        hist.append(tot / max(cnt, 1))
        if log_every and (ep % log_every == 0 or ep == epochs - 1):
            _log(f"epoch {ep}: train mse {hist[-1]:.4e}")
    return fold_standardization(theta.cpu().numpy(), mu, sd, F, H), hist


def save(path, theta, F, H, meta=None):
    path = Path(path)
    path.parent.mkdir(parents=True, exist_ok=True)
    np.savez(path, theta=theta.astype(np.float32), F=np.int64(F), H=np.int64(H),
             meta=np.array(json.dumps(meta or {})))


def load(path=DEFAULT_WEIGHTS):
    d = np.load(path, allow_pickle=False)
    return d["theta"].astype(np.float32), int(d["F"]), int(d["H"]), json.loads(str(d["meta"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--problems", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--width", type=int, default=H_DEFAULT)
    ap.add_argument("--out", default=str(DEFAULT_WEIGHTS))
    a = ap.parse_args()
    from . import kotssn
    ctx = kotssn.Context(0)
    t0 = time.perf_counter()
    X, y, info = build_dataset(ctx, range(a.problems))
    t1 = time.perf_counter()
    ok = sum(1 for i in info if i["status"] == 0)
    _log(f"dataset: {ok}/{len(info)} solved, {X.shape[0]} rows, {t1 - t0:.1f} s, mean iters "
         f"{np.mean([i['iters'] for i in info]):.2f}")
    theta, hist = fit(ctx, X, y, H=a.width, epochs=a.epochs, batch=a.batch, lr=a.lr)
    t2 = time.perf_counter()
    _log(f"training: {t2 - t1:.1f} s, final mse {hist[-1]:.4e}")
    save(a.out, theta, X.shape[1], a.width, dict(problems=a.problems, solved=ok, epochs=a.epochs, batch=a.batch,
                                                 lr=a.lr, final_mse=hist[-1], workload="mix256",
                                                 data_seconds=t1 - t0, train_seconds=t2 - t1))
    ctx.close()
    print(json.dumps(dict(out=a.out, rows=int(X.shape[0]), final_mse=hist[-1], data_s=t1 - t0, train_s=t2 - t1)))


if __name__ == "__main__":
    main()
