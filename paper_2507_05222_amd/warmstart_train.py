#!/usr/bin/env python3
"""Training of the learned warm start of the pressure solve.

Pairs (b, p) come from the plain FP64 path of this library: for seeded cylinder
configurations (Re ~ U[60, 200], wall rotation rate alpha ~ U[0, 2]) on the
2^n x 2^n O-grid, the fractional step is run from uniform flow plus the App. G
perturbation, and every other step from step `first` on the pressure right-hand
side b (exported by the step) and the converged pressure p are block-averaged to
64 x 64. The grid-only operators are built once and shared by all configurations. The network
(qtt_ws_* kernels) maps (b / rms(b), Re / 200, alpha / 2) to p / (rms(b) s0),
where s0 is the training-set mean of rms(p) / rms(b). Held-out configurations
measure the relative L2 error of the coarse prediction.

  python -m paper_2507_05222_amd.warmstart_train --out DIR [--configs 60 --test 12 --steps 28]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def initial_fields(n, A0):
    N = 2 ** n
    i = np.arange(N)
    env = (np.exp((1.0 - (i + 1) / (N + 1)) ** 6) - 1.0) / (np.e - 1.0)
    theta = 2 * np.pi * np.arange(N) / N
    return 1.0 + A0 * env[:, None] * np.sin(theta)[None, :], np.zeros((N, N))


def generate(ctx, n, chi, dt, configs, steps, first, tol, log):
    """Pairs (coarse b, coarse p) of every other step from step `first` on, for each
    configuration, from the library's FP64 path (pressure solved to `tol`)."""
    from paper_2507_05222_amd import flow as F, qtt as Q, warmstart as W
    from qtt_inputs import random_mps_cores
    L = 2 * n
    u0, v0 = initial_fields(n, 1e-2)
    so = lambda t: Q.solve_opts(tol=t, max_sweeps=8, max_local_iters=80, local_tol=1e-2, dtype="f64")
    B, P, C = [], [], []
    base = None
    for ci, (re, alpha) in enumerate(configs):
        t0 = time.perf_counter()
        ops = F.FlowOps(n, 20.0, re, dt, alpha, like=base)
        base = base or ops
        st = F.FlowState(Q.from_dense(ctx, F.grid_to_qtt_order(u0), L, 1e-14, chi, chi),
                         Q.from_dense(ctx, F.grid_to_qtt_order(v0), L, 1e-14, chi, chi),
                         Q.MPS.from_cores(random_mps_cores(L, chi, seed=ci), chi))
        rhs = Q.MPS(L, chi)
        opts = F.step_opts(dt, tol=1e-8, chi=chi, dtype="f64", helm=so(1e-8), pois=so(tol), rhs_out=rhs)
        for s in range(steps):
            F.fractional_step(ctx, ops, st, opts)
            if s >= first and (s - first) % 2 == 0:
                B.append(W.coarse(ctx, rhs))
                P.append(W.coarse(ctx, st.p))
                C.append((re, alpha))
        log(f"config {ci}: Re {re:.1f} alpha {alpha:.2f}, {steps} steps in {time.perf_counter() - t0:.1f}s")
    return np.array(B), np.array(P), np.array(C)


def features(b, c):
    """Network input (3, 64, 64) and the scale rms(b) of one pair (the library's rule)."""
    from paper_2507_05222_amd import warmstart as W
    return W.ws_input(b, c[0], c[1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=10)
    ap.add_argument("--chi", type=int, default=64)
    ap.add_argument("--dt", type=float, default=2e-3)
    ap.add_argument("--configs", type=int, default=60)
    ap.add_argument("--test", type=int, default=12)
    ap.add_argument("--steps", type=int, default=28)
    ap.add_argument("--first", type=int, default=6, help="first step whose pair is kept (then every other step)")
    ap.add_argument("--tol", type=float, default=1e-6, help="pressure tolerance of the data generation")
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=2025)
    ap.add_argument("--pairs", default=None, help="cache of the generated pairs (default OUT/pairs.npz)")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)

    import torch
    from paper_2507_05222_amd import qtt as Q, warmstart as W

    def log(msg):
        print(f"[train] {msg}", flush=True)

    rng = np.random.default_rng(args.seed)
    configs = [(float(rng.uniform(60, 200)), float(rng.uniform(0, 2))) for _ in range(args.configs)]
    ctx = Q.Context(0)
    data = args.pairs or os.path.join(args.out, "pairs.npz")
    if os.path.exists(data):
        z = np.load(data, allow_pickle=False)
        B, P, C = z["b"], z["p"], z["c"]
    else:
        B, P, C = generate(ctx, args.n, args.chi, args.dt, configs, args.steps, args.first, args.tol, log)
        np.savez(data, b=B, p=P, c=C)
    per = len(B) // args.configs
    ntr = (args.configs - args.test) * per
    X, R = zip(*[features(b, c) for b, c in zip(B, C)])
    X, R = np.array(X), np.array(R)
    s0 = float(np.mean([np.sqrt(np.mean(p ** 2)) / r for p, r in zip(P[:ntr], R[:ntr])]))
    Y = np.array([(p / (r * s0))[None] for p, r in zip(P, R)], dtype=np.float32)
    Xg, Yg = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    net = W.Net(ctx, seed=args.seed)

    def test_error():
        out, _ = net.forward(Xg[ntr:], bf16=True)
        o = out.cpu().numpy()
        return float(np.mean([np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(o, Y[ntr:])]))

    log(f"{ntr} training pairs, {len(X) - ntr} held-out; s0 = {s0:.4g}; held-out error before {test_error():.3f}")
    t0 = time.perf_counter()
    for ep in range(args.epochs):
        perm = rng.permutation(ntr)
        lr = args.lr * (0.5 * (1 + np.cos(np.pi * ep / args.epochs)))      # cosine decay
        tot = 0.0
        for i in range(0, ntr - args.batch + 1, args.batch):
            idx = torch.from_numpy(perm[i:i + args.batch]).cuda()
            tot += net.loss_grad(Xg[idx], Yg[idx])
            net.adam(lr)
        if ep % 50 == 0 or ep == args.epochs - 1:
            log(f"epoch {ep}: train mse {tot / max(1, ntr // args.batch):.4g}, held-out rel err {test_error():.3f}")
    secs = time.perf_counter() - t0
    err = test_error()
    W.save(os.path.join(args.out, "wsnet.json"), net.numpy_params(), s0,
           {"train_pairs": int(ntr), "test_pairs": int(len(X) - ntr), "held_out_rel_l2": err, "train_seconds": secs,
            "epochs": args.epochs, "recipe": f"n={args.n} chi={args.chi} dt={args.dt} configs={args.configs} "
                                             f"(held out {args.test}) steps={args.steps} pairs from step "
                                             f"{args.first} every other step, pressure tol {args.tol:g}, "
                                             f"seed={args.seed}; Re~U[60,200], alpha~U[0,2]; taps dilated 1,2,4,8",
            "test_configs": configs[args.configs - args.test:]})
    log(f"done: held-out relative L2 error of the coarse pressure {err:.3f}, training {secs:.1f}s")


if __name__ == "__main__":
    main()
