#!/usr/bin/env python3
"""Benchmark of the QTT fractional step on one MI355X.

Workload: transient cylinder flow on the 2^10 x 2^10 O-grid (20 interleaved
cores, r in [0.5, 20]), Re = 200, dt = 2e-3, bond dimension chi = 64, uniform
inflow plus the seed-0 asymmetric perturbation of amplitude 1e-2 (synthetic
initial data; no dataset). One "step" is one full fractional step (gradients,
convection products, two predictor solves, divergence, pressure solve,
projection) through the C ABI.

Reported: steps/s of the mixed-precision path (BF16 MFMA contractions with FP32
accumulation, FP64 truncation and residuals; Poisson local products in FP32 and
Helmholtz in BF16, both refined against FP64 residuals), the plain FP64 path on
the same GPU, their relative L2 difference, the roofline of the dominant kernel
(HIP events in this process) and the CPU oracle (FD twin, FP64) timed on the
host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}   # dense TFLOP/s, MI355X published


def build_state(Q, F, n, chi, A0, ctx):
    """Initial fields: uniform flow + perturbation, encoded by the library's host TT-SVD."""
    L = 2 * n
    N = 2 ** n
    i = np.arange(N)
    d_eta = 1.0 / (N + 1)
    env = (np.exp((1.0 - (i + 1) * d_eta) ** 6) - 1.0) / (np.e - 1.0)
    theta = 2 * np.pi * np.arange(N) / N
    u = 1.0 + A0 * env[:, None] * np.sin(theta)[None, :]
    v = np.zeros((N, N))
    uq = F.grid_to_qtt_order(u)
    vq = F.grid_to_qtt_order(v)
    U = Q.tt_svd_host(uq, L, 1e-14, chi, chi)
    V = Q.tt_svd_host(vq + 0.0, L, 1e-14, chi, chi)
    return U, V, u, v


def make_p0(Q, L, chi):
    from qtt_inputs import random_mps_cores    # seeded cold start of the first pressure solve
    return Q.MPS.from_cores(random_mps_cores(L, chi, seed=0), chi)


def clone(Q, m):
    c = Q.MPS(m.L, m.cap)
    c.copy_(m)
    return c


def run_path(Q, F, ctx, ops, U0, V0, P0, opts, warmup, steps, timer=None):
    import torch
    st = F.FlowState(clone(Q, U0), clone(Q, V0), clone(Q, P0))
    for _ in range(warmup):
        F.fractional_step(ctx, ops, st, opts)
    torch.cuda.synchronize()
    if timer is not None:
        timer.start()
    t0 = time.perf_counter()
    infos = []
    for s in range(steps):
        infos.append(F.fractional_step(ctx, ops, st, opts))
        print(f"[bench] step {s + 1}/{steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = timer.read() if timer is not None else None
    return st, dt, infos, kt


def dense(Q, F, m, n):
    from paper_2507_05222_amd import flow
    cores = m.cores()
    out = np.ones((1, 1))
    for c in cores:
        out = (out @ c.reshape(c.shape[0], -1)).reshape(-1, c.shape[2])
    q = out.reshape(-1)
    N = 2 ** n
    perm_grid = flow.grid_to_qtt_order(np.arange(N * N, dtype=float).reshape(N, N)).astype(np.int64)
    grid = np.empty(N * N)
    grid[perm_grid] = q
    return grid


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10, help="cores per axis (grid 2^n x 2^n)")
    ap.add_argument("--chi", type=int, default=64)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--timer", default="zip_factor",
                    help="kernel class timed with HIP events for the roofline (dominant kernel)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2507_05222_amd import flow as F, qtt as Q

    n, chi = args.n, args.chi
    L = 2 * n
    Re, dt, A0 = 200.0, 2e-3, 1e-2
    ctx = Q.Context(0)
    t0 = time.perf_counter()
    ops = F.FlowOps(n, 20.0, Re, dt)
    setup_s = time.perf_counter() - t0
    U0, V0, u_init, v_init = build_state(Q, F, n, chi, A0, ctx)
    P0 = make_p0(Q, L, chi)
    tol = 1e-8

    mixed = F.step_opts(dt, tol=tol, chi=chi, dtype="f32", product="bf16",
                        helm=Q.solve_opts(tol=1e-8, max_sweeps=1, max_local_iters=40, local_tol=1e-6, dtype="bf16"),
                        pois=Q.solve_opts(tol=1e-8, max_sweeps=2, max_local_iters=80, local_tol=1e-4, dtype="f32"))
    plain = F.step_opts(dt, tol=tol, chi=chi, dtype="f64",
                        helm=Q.solve_opts(tol=1e-8, max_sweeps=1, max_local_iters=40, local_tol=1e-6, dtype="f64"),
                        pois=Q.solve_opts(tol=1e-8, max_sweeps=2, max_local_iters=80, local_tol=1e-4, dtype="f64"))

    # the timed class and the arithmetic type it runs in on the mixed path
    tdt = {"zip_contract": "f32", "env_gemm": "f32"}.get(args.timer, "f64")
    timer = Q.KernelTimer(ctx, args.timer, tdt) if args.timer != "none" else None
    print("[bench] mixed path", file=sys.stderr, flush=True)
    st_m, t_m, info_m, kt = run_path(Q, F, ctx, ops, U0, V0, P0, mixed, args.warmup, args.steps, timer)
    sps_m = args.steps / t_m

    res = {}
    sps_p = None
    if not args.no_fp64:
        k64 = args.fp64_steps or args.steps
        print("[bench] fp64 path", file=sys.stderr, flush=True)
        st_p, t_p, info_p, _ = run_path(Q, F, ctx, ops, U0, V0, P0, plain, args.warmup, k64)
        sps_p = k64 / t_p
        if k64 == args.steps:
            for name in ("u", "v", "p"):
                a = dense(Q, F, getattr(st_m, name), n)
                b = dense(Q, F, getattr(st_p, name), n)
                res[name] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

    cpu = None
    if not args.no_cpu:
        from oracle import fd
        from oracle.grid import OGrid
        g = OGrid(n, n)
        S = fd.FDSolver(g, Re, dt, solver="fft")
        u, v = u_init.ravel().copy(), v_init.ravel().copy()
        u, v, _ = S.step(u, v)          # warm-up (first-touch of the operators)
        ns, t1 = 0, time.perf_counter()
        while time.perf_counter() - t1 < 15.0 and ns < args.steps + args.warmup:
            u, v, _ = S.step(u, v)
            ns += 1
        tc = time.perf_counter() - t1
        cpu = {"value": ns / tc, "unit": "steps/s", "cores": 1, "kind": "oracle",
               "sample": f"{ns} FD steps (FP64, FFT/Thomas solves) on the same 2^{n}x2^{n} grid and initial field"}

    roof = None
    if kt is not None and kt["launches"] > 0:
        ach = kt["flops"] / (kt["ms"] * 1e-3) / 1e12
        alu = kt["name"] in ("zip_factor", "rl_svd", "qr_moves", "cg_update")
        peak = 78.6 if alu else PEAKS[kt["dtype"]]    # FP64 vector ALU peak for the factorisations
        roof = {"bound": "alu" if alu else "mfma", "achieved": round(ach, 4), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 6), "traffic": None, "kernel": kt["name"],
                "avg_launch_us": round(1e3 * kt["ms"] / kt["launches"], 3), "launches": kt["launches"],
                "flops_per_launch": kt["flops"] / kt["launches"],
                "bytes_per_launch": kt["bytes"] / kt["launches"]}

    out = {
        "metric": "QTT fractional steps/s at 2^20 grid, chi=64: mixed+warm-start vs FP64, same error",
        "value": round(sps_m, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_m / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": f"cylinder O-grid 2^{n}x2^{n} ({L} interleaved cores), chi={chi}, Re={Re:g}, "
                               f"dt={dt:g}, perturbation A0={A0:g}; Poisson initial guess = previous pressure",
                   "fp64_steps_per_s": None if sps_p is None else round(sps_p, 4),
                   "speedup_vs_fp64": None if sps_p is None else round(sps_m / sps_p, 3),
                   "mixed_vs_fp64_rel_l2": res or None,
                   "poisson_residual_last": info_m[-1].poisson.residual if info_m else None,
                   "poisson_cg_iters_last": info_m[-1].poisson.local_iters if info_m else None,
                   "setup_s": round(setup_s, 2)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
