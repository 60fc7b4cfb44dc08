"""Train the learned warm start (the network of eodabe_set_predictor) on the
GPU with the library's own forward, backward and Adam kernels.

    python -m paper_2506_22713_amd.train_predictor --out paper_2506_22713_amd/predictor.ckpt

Training set: seeded matrices from the spectrum generator (geometric,
polynomial and stepped singular-value decay) and the image generator of
workloads/, at log-uniform sizes (256 .. 4096 rows) and tolerances.  Label:
the rank the plain loop returns (eodabe_basis); inputs: its first 64
stopping-test values and the test's threshold eps = tol ||A||_F
(eodabe_mlp_features).  Matrices of rank below 64 are
left out: their first 64 columns already stop the loop and the predictor is
never consulted.  --resume continues from a checkpoint (Adam state and step
included).
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np
import torch

import paper_2506_22713_amd as E
from paper_2506_22713_amd import predictor as PR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
import workloads as W  # noqa: E402

BLOCK = 32


def log(*a):
    print("[train]", *a, file=sys.stderr, flush=True)


def logu(rng, lo, hi):
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def make_sample(seed: int):
    """(A on the device, tol, dtype, description) of training sample `seed`."""
    rng = np.random.default_rng([seed, 17])
    kind = rng.choice(["geom", "poly", "stairs", "image"], p=[0.4, 0.25, 0.15, 0.2])
    if kind == "image":
        size = int(logu(rng, 512, 2048))
        noise = logu(rng, 0.005, 1.0)
        tol = logu(rng, 1e-4, 1e-2)
        A = torch.from_numpy(W.image(int(rng.integers(1 << 30)), size, noise)).cuda()
        return A, tol, torch.float32, f"image {size} noise {noise:.3g}"
    m = int(logu(rng, 256, 4096))
    n = int(logu(rng, 128, m))
    r = int(min(logu(rng, 40, 700), n))
    param = {"geom": rng.uniform(0.5, 10.0), "poly": rng.uniform(0.3, 3.0), "stairs": rng.integers(4, 40)}[kind]
    sig = W.spectrum_sigma(kind, r, float(param))
    tol = logu(rng, 1e-7, 1e-2)
    dtype = torch.float64 if tol < 1e-5 else torch.float32
    noise = logu(rng, 1e-12, 1e-3) * float(np.sqrt(np.sum(sig ** 2) / (m * n)))
    A = W.spectrum_torch(int(rng.integers(1 << 30)), m, n, sig, noise, dtype=dtype)
    return A, tol, dtype, f"{kind} {m}x{n} r{r} p{float(param):.3g}"


def label(A: torch.Tensor, tol: float, dtype, seed: int):
    """(rank, first 64 stopping-test values, eps) of the plain loop."""
    Q, d, info = E.basis(A, tol, block=BLOCK, seed=seed, dtype=dtype)
    return int(info.rank), d, float(info.eps)


def build_set(count: int, first_seed: int):
    X, T, desc = [], [], []
    seed = first_seed
    t0 = time.time()
    while len(X) < count:
        A, tol, dtype, what = make_sample(seed)
        m, n = A.shape
        r, d, eps = label(A, tol, dtype, seed)
        seed += 1
        if r < 64 or d.size < 64:
            continue
        X.append(PR.features(d[:64], m, n, eps))
        T.append(math.log1p(r))
        desc.append((what, m, n, tol, r))
        if len(X) % 250 == 0:
            log(f"{len(X)} samples ({seed - first_seed} drawn, {time.time() - t0:.0f} s)")
    return np.stack(X), np.asarray(T, dtype=np.float32), desc


def coverage(pred: PR.Predictor, ctx, X, T, margin: float):
    """Fraction of samples whose warm-start width d0 holds the rank (no
    fallback), mean surplus blocks (d0 - rank - 1) / b, and the MSE of head 0."""
    Y = pred.forward(ctx, torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    ranks = np.expm1(T.astype(np.float64))
    d0 = np.array([BLOCK * max(1, math.ceil(((math.exp(y1) - 1) * (1 + margin) + 1) / BLOCK)) for y1 in Y[:, 1]])
    hit = d0 > ranks
    surplus = np.where(hit, (d0 - ranks - 1) / BLOCK, 0.0)
    return float(hit.mean()), float(surplus.mean()), float(np.mean((Y[:, 0] - T) ** 2))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=3000)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--margin", type=float, default=0.1)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "predictor.ckpt"))
    ap.add_argument("--resume", default=None)
    args = ap.parse_args(argv)
    ctx = E.Context()
    log("building the training set")
    X, T, desc = build_set(args.samples, 1_000_000 * (args.seed + 1))
    nv = max(len(X) // 7, 1)
    perm = np.random.default_rng(args.seed).permutation(len(X))
    Xv, Tv, Xt, Tt = X[perm[:nv]], T[perm[:nv]], X[perm[nv:]], T[perm[nv:]]
    pred = PR.Predictor.load(args.resume) if args.resume else PR.Predictor(seed=args.seed)
    Xd, Td = torch.from_numpy(Xt).cuda(), torch.from_numpy(Tt).cuda()
    steps_per_epoch = max(1, math.ceil(len(Xt) / args.batch))
    total = args.epochs * steps_per_epoch
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed)
    log(f"training on {len(Xt)} samples, validating on {len(Xv)}; {total} steps")
    k = 0
    for ep in range(args.epochs):
        order = torch.randperm(len(Xt), generator=g, device="cuda")
        for s in range(steps_per_epoch):
            idx = order[s * args.batch:(s + 1) * args.batch]
            lr = args.lr * 0.5 * (1 + math.cos(math.pi * k / total))      # cosine decay
            loss = pred.train_step(ctx, Xd[idx], Td[idx], lr)
            k += 1
        if ep % 50 == 0 or ep == args.epochs - 1:
            hit, sur, mse = coverage(pred, ctx, Xv, Tv, args.margin)
            log(f"epoch {ep}: train loss {loss:.4f}  val mse(log1p rank) {mse:.4f}  "
                f"no-fallback {hit:.3f}  surplus blocks {sur:.2f}")
    hit, sur, mse = coverage(pred, ctx, Xv, Tv, args.margin)
    pred.save(args.out, meta=dict(samples=len(X), val=len(Xv), block=BLOCK, margin=args.margin,
                                  val_mse_log1p_rank=mse, val_no_fallback=hit, val_surplus_blocks=sur,
                                  epochs=args.epochs, lr=args.lr, seed=args.seed))
    log(f"saved {args.out}: val no-fallback {hit:.3f}, surplus {sur:.2f} blocks, mse {mse:.4f}")
    print(dict(val_no_fallback=hit, val_surplus_blocks=sur, val_mse=mse, samples=len(X)), flush=True)


if __name__ == "__main__":
    main()
