#!/usr/bin/env python3
"""Benchmark of the QTT fractional step on one MI355X.

Workload: transient cylinder flow on the 2^10 x 2^10 O-grid (20 interleaved
cores, r in [0.5, 20]), Re = 200, dt = 2e-3, bond dimension chi = 64, uniform
inflow plus the asymmetric App. G perturbation of amplitude 1e-2 (synthetic
initial data; no dataset). One "step" is one full fractional step (gradients,
convection products, two predictor solves, divergence, pressure solve,
projection) through the C ABI, inputs resident on the GPU.

Two paths from the same initial state, both solving the predictor and pressure
systems to the same residual tolerance (default 1e-8):
  plain -- FP64 throughout, the previous pressure as the start of the pressure solve;
  mixed -- FP64 fits, FP32-MFMA Hadamard products, the learned warm start of the
           pressure solve (the network's guess or the previous pressure, whichever
           the solve's energy rates lower).
Both are scored against the FP64 FD oracle after the same number of steps by the
|J|-weighted relative L2 error of u, v, p (Sec. 4); `value` is the mixed path's
rate if all three errors are within 3e-3, else the plain path's, and
config.reported_path says which. The oracle run is the CPU-baseline leg. The
roofline entry is the dominant kernel (the one-launch local CG), measured with HIP
events on the library's stream during one extra step.
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
TRAFFIC = os.path.join(ROOT, "profiles", "k_cg_coop_cylinder_2e20_chi64_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2507_05222_amd", "csrc", f) for f in ("solve.hip", "device_common.h")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_profile():
    """From the committed rocprofv3 summaries of the dominant kernel: HBM bytes per
    launch (--pmc FETCH_SIZE and WRITE_SIZE, scaled by what they read for a plain
    copy) and the kernel-trace average duration; None when the kernel sources
    changed since the counters were taken."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return {"traffic": 1024.0 * (t["fetch_kib_per_dispatch"] * t["fetch_factor"] +
                                 t["write_kib_per_dispatch"] * t["write_factor"]),
            "trace_avg_us": t.get("kernel_trace_avg_us")}


def initial_fields(n, A0):
    """Uniform flow u = 1, v = 0 plus the App. G modulation of u (grid order), with
    the envelope read as vanishing towards the far field (row N-1)."""
    N = 2 ** n
    i = np.arange(N)
    d_eta = 1.0 / (N + 1)
    env = (np.exp((1.0 - (i + 1) * d_eta) ** 6) - 1.0) / (np.e - 1.0)
    theta = 2 * np.pi * np.arange(N) / N
    u = 1.0 + A0 * env[:, None] * np.sin(theta)[None, :]
    return u, np.zeros((N, N))


def clone(Q, m):
    c = Q.MPS(m.L, m.cap)
    c.copy_(m)
    return c


def dense(Q, F, m, n, order="interleaved"):
    cores = m.cores()
    out = np.ones((1, 1))
    for c in cores:
        out = (out @ c.reshape(c.shape[0], -1)).reshape(-1, c.shape[2])
    q = out.reshape(-1)
    N = 2 ** n
    perm = F.grid_to_qtt_order(np.arange(N * N, dtype=float).reshape(N, N), order).astype(np.int64)
    grid = np.empty(N * N)
    grid[perm] = q
    return grid.reshape(N, N)


def exact_rel_error(Q, ctx, M_cores, x, y):
    """||y - M x|| / ||M x|| from exact FP64 TT inner products on the GPU:
    <y, y> - 2 <y, M x> + <x, (M^T M) x>, with M^T M assembled core by core as an MPO
    of bond w^2 (no dense vectors at L = 24)."""
    N = []
    for c in M_cores:                      # c[a][r'][r][b], r' the output index
        a, _, _, b = c.shape
        n = np.einsum("aisb,citd->acstbd", c, c).reshape(a * a, 2, 2, b * b)
        N.append(n)
    nn = Q.dot_mpo(ctx, [x], [Q.MPO.from_cores(N)], [x])[0]
    ym = Q.dot_mpo(ctx, [y], [Q.MPO.from_cores(M_cores)], [x])[0]
    yy = Q.dot(ctx, [y], [y])[0]
    return float(np.sqrt(max(nn - 2.0 * ym + yy, 0.0) / nn))


def left_canonical(cores):
    """Input preparation of the kernel sweep: the random cores made left-orthonormal by
    host QR from the left (the last core keeps the norm); the bonds do not change."""
    out, carry = [], None
    for k, c in enumerate(cores):
        if carry is not None:
            c = np.tensordot(carry, c, axes=(1, 0))
        a, d, b = c.shape
        if k == len(cores) - 1:
            out.append(c)
            break
        q, r = np.linalg.qr(c.reshape(a * d, b))
        out.append(q.reshape(a, d, q.shape[1]))
        carry = r
    return out


def sweep(args):
    """Isolated kernel sweep: random MPS (L = 24, cores N(0, 1/chi), then left-canonical) times random MPO
    (bond w, entries N(0, 1)), zip-up apply plus rounding to chi, `trials` chains per
    call. Reports the whole call's time over all chains (the library runs batches of 32
    chains up to four at a time), the site contractions in TFLOP/s from the library's
    work counters and HIP-event brackets over one batch of (at most) 32 chains, where no
    other batch runs beside them, and, for FP64, the truncation error ||y - M x|| / ||M x||
    of the first chain from exact inner products. In FP64 at slot capacity 64 or 128 both
    contractions of a site run in one kernel (k_zip_fused, reported under carry_x_core,
    "fused": true); otherwise k_zip_t1 (carry_x_core) and k_zip_t2 (x_mpo_core)."""
    import torch
    from paper_2507_05222_amd import qtt as Q
    from qtt_inputs import random_mps_cores, random_mpo_cores
    L = 24
    ctx = Q.Context(0)
    for chi in [int(c) for c in args.sweep_chi.split(",")]:
        xs = [Q.MPS.from_cores(left_canonical(random_mps_cores(L, chi, seed=100 + t)), chi)
              for t in range(args.trials)]
        for w in [int(v) for v in args.sweep_w.split(",")]:
            Ms = [Q.MPO.from_cores(random_mpo_cores(L, w, seed=200 + t)) for t in range(args.trials)]
            ys = [Q.MPS(L, chi) for _ in range(args.trials)]
            for dt in args.sweep_dtypes.split(","):
                Q.apply_mpo(ctx, Ms, xs, ys, tol=0.0, chi=chi, dtype=dt, fit=0)      # warm-up
                torch.cuda.synchronize()
                rec = {"sweep": "apply+round", "L": L, "chi": chi, "w": w, "dtype": dt, "trials": args.trials}
                t0 = time.perf_counter()
                Q.apply_mpo(ctx, Ms, xs, ys, tol=0.0, chi=chi, dtype=dt, fit=0)
                torch.cuda.synchronize()
                rec["apply_ms"] = round(1e3 * (time.perf_counter() - t0), 3)
                rec["chains_per_s"] = round(args.trials / (rec["apply_ms"] * 1e-3), 2)
                nb = min(args.trials, 32)
                rec["kernel_rates_chains"] = nb
                for cls, tag in (("zip_contract", "carry_x_core"), ("zip_mpo", "x_mpo_core")):
                    timer = Q.KernelTimer(ctx, cls, dt)
                    timer.start()
                    Q.apply_mpo(ctx, Ms[:nb], xs[:nb], ys[:nb], tol=0.0, chi=chi, dtype=dt, fit=0)
                    torch.cuda.synchronize()
                    kt = timer.read()
                    tf = kt["flops"] / (kt["ms"] * 1e-3) / 1e12 if kt["ms"] > 0 else 0.0
                    rec[tag] = {"tflops": round(tf, 3), "frac_of_peak": round(tf / PEAKS[dt], 5),
                                "launches": kt["launches"], "avg_us": round(1e3 * kt["ms"] / max(kt["launches"], 1), 2),
                                "gflop": round(kt["flops"] / 1e9, 3),
                                "alg_gb_s": round(kt["bytes"] / (kt["ms"] * 1e-3) / 1e9, 1) if kt["ms"] > 0 else None}
                a, b = rec["carry_x_core"], rec["x_mpo_core"]
                tot_ms = (a["launches"] * a["avg_us"] + b["launches"] * b["avg_us"]) * 1e-3
                tf = (a["gflop"] + b["gflop"]) / max(tot_ms, 1e-9)
                rec["contraction"] = {"tflops": round(tf, 3), "frac_of_peak": round(tf / PEAKS[dt], 5)}
                rec["fused"] = b["launches"] == 0 and a["launches"] > 0
                if dt == "f64":
                    # M^T M has bond w^2; the library's MPO bond limit is 512
                    rec["trunc_rel_err_trial0"] = (exact_rel_error(Q, ctx, random_mpo_cores(L, w, seed=200), xs[0],
                                                                   ys[0]) if w * w <= 512 else None)
                if rec["fused"]:
                    # the fused kernel per site: work from the actual bonds (the zip-up's
                    # output bonds are those of y, which the final sweep at tol 0 keeps),
                    # time from the per-launch brackets of the last timed apply of class 0
                    timer = Q.KernelTimer(ctx, "zip_contract", dt)
                    timer.start()
                    Q.apply_mpo(ctx, Ms[:nb], xs[:nb], ys[:nb], tol=0.0, chi=chi, dtype=dt, fit=0)
                    timer.read()
                    per = timer.durations()
                    xb = [min(2 ** k, 2 ** (L - k), chi) for k in range(L + 1)]
                    yb = ys[0].bonds()
                    wb = [1] + [w] * (L - 1) + [1]
                    sat = [k for k in range(L) if xb[k] == chi and xb[k + 1] == chi]
                    fl = sum(nb * (4.0 * yb[k] * wb[k] * xb[k + 1] * xb[k] +
                                            8.0 * yb[k] * wb[k + 1] * xb[k + 1] * wb[k]) for k in sat)
                    ms = sum(per[k] for k in sat)
                    tfs = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
                    rec["contraction_saturated_sites"] = {"sites": [sat[0], sat[-1]] if sat else [],
                                                          "tflops": round(tfs, 3),
                                                          "frac_of_peak": round(tfs / PEAKS[dt], 5),
                                                          "avg_us": round(1e3 * ms / max(len(sat), 1), 2)}
                print(json.dumps(rec), flush=True)
            del Ms, ys
            torch.cuda.empty_cache()


CASES = {
    # transient cylinder of the C3 workload: 2^10 x 2^10, r_out 20, App. G perturbation 1e-2
    "c3": dict(n=10, r_out=20.0, Re=200.0, alpha=0.0, dt=2e-3, A0=1e-2, chi=64),
    # the paper's rotating cylinder (Sec. 4.2, Table 2): G1 = 2^8 x 2^8, outer diameter
    # 32 D, Re = 100, rotation rate 1 (Eq. rot_bc), dt = 2e-3, uniform start
    "rotating_g1": dict(n=8, r_out=16.0, Re=100.0, alpha=1.0, dt=2e-3, A0=0.0, chi=40),
}


def shedding(args):
    """A long transient run (--case: "c3", the 2^10 x 2^10 transient cylinder, or
    "rotating_g1", the paper's rotating cylinder of Table 2; --chi-case overrides the
    case's bond; FP64 throughout, or with --shedding-product f32 the mixed path's FP32
    Hadamard products), drag and lift every 10 steps, resumable: the TT
    state, the step count and the force history go to --ckpt-out after every 1000
    steps and are read from --ckpt-in if given. Once --shedding-steps are done the
    Strouhal number, lift amplitude and mean lift (upward zero crossings of C_L, last
    half of the run) are printed as one JSON line."""
    import torch
    from paper_2507_05222_amd import diag as D, flow as F, qtt as Q
    from qtt_inputs import random_mps_cores
    c = dict(CASES[args.case])
    if args.chi_case:
        c["chi"] = args.chi_case
    n, chi, Re, dt, A0 = c["n"], c["chi"], c["Re"], c["dt"], c["A0"]
    L = 2 * n
    ctx = Q.Context(0)
    ops = F.FlowOps(n, c["r_out"], Re, dt, c["alpha"])
    so = lambda tol, sw: Q.solve_opts(tol=tol, max_sweeps=sw, max_local_iters=80, local_tol=args.local_tol, dtype="f64")
    opts = F.step_opts(dt, tol=1e-8, chi=chi, dtype="f64", product=args.shedding_product, helm=so(1e-8, 4),
                       pois=so(args.pois_tol, 8))
    st = F.FlowState(Q.MPS(L, chi), Q.MPS(L, chi), Q.MPS(L, chi))
    if args.ckpt_in and os.path.exists(args.ckpt_in):
        z = np.load(args.ckpt_in, allow_pickle=False)
        for k in ("u", "v", "p"):
            getattr(st, k).data.copy_(torch.from_numpy(z[k + "_data"]))
            getattr(st, k).bond.copy_(torch.from_numpy(z[k + "_bond"]))
        done, hist = int(z["step"]), [tuple(r) for r in z["hist"]]
    else:
        u0, v0 = initial_fields(n, A0)
        for k, f in (("u", u0), ("v", v0)):
            getattr(st, k).copy_(Q.from_dense(ctx, F.grid_to_qtt_order(f), L, 1e-14, chi, chi))
        st.p.copy_(Q.MPS.from_cores(random_mps_cores(L, chi, seed=0), chi))
        done, hist = 0, []

    def save():
        if args.ckpt_out:
            np.savez(args.ckpt_out, step=done, hist=np.array(hist if hist else np.zeros((0, 3))),
                     **{k + "_data": getattr(st, k).data.cpu().numpy() for k in ("u", "v", "p")},
                     **{k + "_bond": getattr(st, k).bond.cpu().numpy() for k in ("u", "v", "p")})

    total = args.shedding_steps
    end = min(total, done + args.steps_per_call)
    t0 = time.perf_counter()
    s0 = done
    while done < end:
        F.fractional_step(ctx, ops, st, opts)
        done += 1
        if done % 10 == 0:
            cd, cl = D.forces(ctx, ops.cyl, st.u, st.v, st.p)
            hist.append((done, cd, cl))
        if done % 1000 == 0 or done == end:
            torch.cuda.synchronize()
            save()
        if done % 250 == 0 or done == end:
            print(f"[bench] {args.case} step {done}/{total} t {done * dt:.2f} C_D {hist[-1][1]:.5f} "
                  f"C_L {hist[-1][2]:.3e} {(done - s0) / (time.perf_counter() - t0):.2f} steps/s",
                  file=sys.stderr, flush=True)
    out = {"workload": f"{args.case}: Re={Re:g}, rotation rate {c['alpha']:g}, O-grid 2^{n}x2^{n}, "
                       f"r_out={c['r_out']:g}, chi={chi}, dt={dt:g}, A0={A0:g}",
           "steps_done": done, "steps_total": total,
           "steps_per_s_this_call": round((done - s0) / (time.perf_counter() - t0), 3)}
    if done >= total and hist:
        h = np.array(hist)
        St, amp = D.strouhal(h[:, 0] * dt, h[:, 2])
        half = h[len(h) // 2:]
        out.update({"St": St, "lift_amplitude": amp, "C_L_mean_last_half": float(half[:, 2].mean()),
                    "C_D_mean_last_half": float(half[:, 1].mean())})
    print(json.dumps(out), flush=True)


def steady(args):
    """Steady cylinder flow, Re = 40, O-grid 2^8 x 2^8 (16 cores), chi = 32, dt = 5e-3:
    the same run with FP64 and with FP32-MFMA contractions (fits and Hadamard
    products; FP64 solves), drag and lift from the library's diagnostics. The
    CPU-baseline leg runs the FD oracle over the same steps; its fields and forces
    score both runs."""
    import torch
    from paper_2507_05222_amd import diag as D, flow as F, qtt as Q
    from qtt_inputs import random_mps_cores
    n, chi, Re, dt, K = 8, args.steady_chi, 40.0, 5e-3, args.steady_steps
    L = 2 * n
    ctx = Q.Context(0)
    ops = F.FlowOps(n, 20.0, Re, dt)
    u0, v0 = initial_fields(n, 1e-2)
    so = lambda tol: Q.solve_opts(tol=tol, max_sweeps=8, max_local_iters=80, local_tol=1e-2, dtype="f64")
    res = {}
    for name, dtype in (("fp64", "f64"), ("fp32", "f32")):
        if name not in args.steady_paths.split(","):
            continue
        st = F.FlowState(Q.tt_svd_host(F.grid_to_qtt_order(u0), L, 1e-14, chi, chi),
                         Q.tt_svd_host(F.grid_to_qtt_order(v0), L, 1e-14, chi, chi),
                         Q.MPS.from_cores(random_mps_cores(L, chi, seed=0), chi))
        opts = F.step_opts(dt, tol=1e-8, chi=chi, dtype=dtype, product=dtype, helm=so(1e-8), pois=so(1e-7))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = []
        for s_ in range(K):
            F.fractional_step(ctx, ops, st, opts)
            if (s_ + 1) % 100 == 0:
                hist.append(D.forces(ctx, ops.cyl, st.u, st.v, st.p))
                print(f"[bench] steady {name} step {s_ + 1}/{K} C_D {hist[-1][0]:.5f} C_L {hist[-1][1]:.2e}",
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        res[name] = {"steps_per_s": round(K / (time.perf_counter() - t0), 3),
                     "C_D": hist[-1][0], "C_L": hist[-1][1],
                     "fields": {k: dense(Q, F, getattr(st, k), n) for k in ("u", "v", "p")}}
    cpu = None
    if not args.no_cpu:
        from oracle import diag, fd
        from oracle.grid import OGrid
        g = OGrid(n, n)
        S = fd.FDSolver(g, Re, dt, solver="fft")
        u, v = u0.ravel().copy(), v0.ravel().copy()
        t1 = time.perf_counter()
        for s_ in range(K):
            ref = S.step(u, v, return_stages=True)
            u, v = ref["u"], ref["v"]
        tc = time.perf_counter() - t1
        bc = fd.velocity_bc(g, 0.0)
        cd, cl = diag.forces(g, ref["u"], ref["v"], ref["p"], Re, bc["u_wall"], bc["v_wall"])
        cpu = {"value": round(K / tc, 3), "unit": "steps/s", "cores": 1, "kind": "oracle",
               "sample": f"{K} FD steps on the same 2^{n}x2^{n} grid", "C_D": cd, "C_L": cl}
        for r in res.values():
            f = r["fields"]
            r["eps_l2_vs_oracle"] = {k: diag.eps_l2(g, f[k].ravel(), ref[k]) for k in ("u", "v", "p")}
            r["C_D_rel_err"] = abs(r["C_D"] - cd) / abs(cd)
            r["C_L_abs_err"] = abs(r["C_L"] - cl)
    for r in res.values():
        r.pop("fields")
    print(json.dumps({"workload": f"steady cylinder Re={Re:g}, O-grid 2^{n}x2^{n}, chi={chi}, dt={dt:g}, {K} steps",
                      "paths": res, "cpu_baseline": cpu}), flush=True)


def exact_product_cores(mpo_cores, mps_cores):
    """Cores of M x with fused bonds (Sec. 2.1.2), no truncation: core k is
    sum_r M_k[a][r'][r][b] x_k[c][r][d] with left bond (a, c) and right bond (b, d)."""
    prod = []
    for m, c in zip(mpo_cores, mps_cores):
        a, _, _, bw = m.shape
        cl, _, cr = c.shape
        prod.append(np.einsum("aosb,csd->acobd", m, c).reshape(a * cl, 2, bw * cr))
    return prod


def global_residual(Q, ctx, A, x, b):
    """||A x - b|| / ||b|| of a solve in TT form, without the cancellation of the expanded
    form <x, A^T A x> - 2 <b, A x> + <b, b>. A x is formed exactly, core by core (the
    mat-vec with fused bond of Sec. 2.1.2, bond w chi, built here on the host as a read-out
    of the result, not a step of the method), A x - b is rounded by the library from the
    explicit direct sum (Householder QR and Jacobi SVD sweeps, backward stable: the error
    is of the order of the rounding of the terms, not of their difference), and its norm
    is read. Needs w chi + cap(b) <= 512."""
    prod = exact_product_cores(A.cores(), x.cores())
    cap = max(max(p.shape[0], p.shape[2]) for p in prod)
    ax = Q.MPS.from_cores(prod, cap)
    r = Q.MPS(x.L, cap + b.cap)
    Q.add(ctx, 1.0, [ax], -1.0, [b], [r], tol=1e-13, chi=cap + b.cap)
    rr = float(Q.dot(ctx, [r], [r])[0])
    bb = float(Q.dot(ctx, [b], [b])[0])
    return float(np.sqrt(max(rr, 0.0) / bb))


def run_path(Q, F, ctx, ops, U0, V0, P0, opts, warmup, steps, tag):
    import torch
    st = F.FlowState(clone(Q, U0), clone(Q, V0), clone(Q, P0))
    for _ in range(warmup):
        F.fractional_step(ctx, ops, st, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for s in range(steps):
        infos.append(F.fractional_step(ctx, ops, st, opts))
        if (s + 1) % 20 == 0 or s + 1 == steps:
            print(f"[bench] {tag} step {s + 1}/{steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return st, time.perf_counter() - t0, infos


def _oracle_ensemble(args_tuple):
    """One independent FD oracle flow (CPU baseline ensemble worker): steps/s."""
    n, Re, dt, A0, steps, seed = args_tuple
    import numpy as np
    from oracle import fd
    from oracle.grid import OGrid
    g = OGrid(n, n)
    S = fd.FDSolver(g, Re, dt, solver="fft")
    u, v = fd.uniform_flow(g)
    u = u + fd.perturbation(g, A0 * (1.0 + 0.1 * seed))
    t0 = time.perf_counter()
    for _ in range(steps):
        u, v, _p = S.step(u, v)
    return steps / (time.perf_counter() - t0)


def cpu_baseline(args, n, Re, dt, A0, u_init, v_init, nsteps):
    """The FP64 FD oracle (FFT-in-xi / Thomas-in-eta solves) on the same grid and initial
    field for the same number of steps: its fields score the GPU paths. Its step is
    single-threaded (numpy FFT, scipy CSR products, the Thomas recurrence), so one flow
    uses one core; an ensemble of independent flows, one per process, shows the host's
    throughput on 8 and on all of its cores."""
    from oracle import fd
    from oracle.grid import OGrid
    g = OGrid(n, n)
    S = fd.FDSolver(g, Re, dt, solver="fft")
    u, v = u_init.ravel().copy(), v_init.ravel().copy()
    t1 = time.perf_counter()
    for _ in range(nsteps):
        ref = S.step(u, v, return_stages=True)
        u, v = ref["u"], ref["v"]
    tc = time.perf_counter() - t1
    host = os.cpu_count() or 1
    cpu = {"value": round(nsteps / tc, 4), "unit": "steps/s", "cores": 1, "kind": "oracle", "host_cores": host,
           "sample": f"{nsteps} FD steps of one flow (FP64; FFT-in-xi / Thomas-in-eta pressure and Helmholtz "
                     f"solves) on the same 2^{n}x2^{n} grid and initial field; single-threaded"}
    if args.cpu_ensemble > 0:
        import multiprocessing as mp
        ens = {}
        for procs in sorted({min(8, host), host}):
            with mp.get_context("spawn").Pool(procs) as pool:
                rates = pool.map(_oracle_ensemble, [(n, Re, dt, A0, args.cpu_ensemble, i) for i in range(procs)])
            ens[str(procs)] = round(float(sum(rates)), 3)
        cpu["ensemble_steps_per_s"] = ens
        cpu["ensemble_note"] = (f"independent flows, one per process, {args.cpu_ensemble} steps each: aggregate "
                                f"steps/s of the host with 8 and with all {host} cores")
    return g, ref, cpu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=10, help="cores per axis (grid 2^n x 2^n)")
    ap.add_argument("--chi", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-8,
                    help="residual tolerance of the pressure and predictor solves, the same for both paths")
    ap.add_argument("--local-tol", type=float, default=1e-2,
                    help="local CG stop of the solves: reduction of each local residual")
    ap.add_argument("--product", default="f32", help="MFMA type of the mixed path's Hadamard products")
    ap.add_argument("--no-learned", action="store_true", help="mixed path without the learned warm start")
    ap.add_argument("--order", default="interleaved", choices=["interleaved", "concatenated"],
                    help="bit order of the fields and operators (the learned warm start needs interleaved)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-ensemble", type=int, default=20,
                    help="steps per process of the CPU ensemble measurement (0: skip)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="isolated MPO x MPS apply + round sweep instead of the step benchmark (one JSON line per shape)")
    ap.add_argument("--sweep-chi", default="64,128,256")
    ap.add_argument("--no-residual", action="store_true",
                    help="skip the global residual read-out after the timed steps (several seconds of "
                         "rounding at bond 448; kernel traces of the step leave it out)")
    ap.add_argument("--sweep-w", default="5,15,30")
    ap.add_argument("--sweep-dtypes", default="f64,f32,bf16")
    ap.add_argument("--trials", type=int, default=32, help="independent chains per apply call in the sweep")
    ap.add_argument("--steady", action="store_true",
                    help="steady cylinder Re=40 on 2^8 x 2^8, chi 32: FP64 vs FP32-MFMA contractions, forces vs the oracle")
    ap.add_argument("--steady-steps", type=int, default=2000)
    ap.add_argument("--steady-chi", type=int, default=32, help="bond of the --steady run")
    ap.add_argument("--steady-paths", default="fp64,fp32", help="paths of the --steady run (fp64, fp32)")
    ap.add_argument("--shedding", action="store_true",
                    help="long transient run (--case c3 or rotating_g1) on the FP64 path, forces every 10 steps, resumable")
    ap.add_argument("--shedding-steps", type=int, default=20000)
    ap.add_argument("--case", default="c3", choices=["c3", "rotating_g1"], help="case of the --shedding run")
    ap.add_argument("--chi-case", type=int, default=0, help="bond of the --shedding run (0: the case's)")
    ap.add_argument("--steps-per-call", type=int, default=20000)
    ap.add_argument("--ckpt-in", default=None)
    ap.add_argument("--ckpt-out", default=None)
    ap.add_argument("--shedding-product", default="f64", choices=["f64", "f32", "bf16"],
                    help="MFMA type of the Hadamard products of the --shedding run")
    ap.add_argument("--pois-tol", type=float, default=1e-8, help="pressure tolerance of the --shedding run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this library is measured on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    if args.sweep:
        sweep(args)
        return
    if args.steady:
        steady(args)
        return
    if args.shedding:
        shedding(args)
        return

    import torch
    from paper_2507_05222_amd import flow as F, qtt as Q, warmstart as W

    n, chi = args.n, args.chi
    L = 2 * n
    Re, dt, A0, alpha = 200.0, 2e-3, 1e-2, 0.0
    ctx = Q.Context(0)
    t0 = time.perf_counter()
    ops = F.FlowOps(n, 20.0, Re, dt, alpha, order=args.order)
    setup_s = time.perf_counter() - t0
    u_init, v_init = initial_fields(n, A0)
    U0 = Q.from_dense(ctx, F.grid_to_qtt_order(u_init, args.order), L, 1e-14, chi, chi)
    V0 = Q.from_dense(ctx, F.grid_to_qtt_order(v_init, args.order), L, 1e-14, chi, chi)
    from qtt_inputs import random_mps_cores     # seeded cold start of the first pressure solve
    P0 = Q.MPS.from_cores(random_mps_cores(L, chi, seed=0), chi)

    def so(sweeps):
        return Q.solve_opts(tol=args.tol, max_sweeps=sweeps, max_local_iters=80, local_tol=args.local_tol,
                            dtype="f64")

    # plain: FP64 throughout; mixed: FP64 fits (their errors feed the divergence),
    # Hadamard products on FP32 (or BF16) MFMA, learned warm start of the pressure solve
    plain = F.step_opts(dt, tol=1e-8, chi=chi, dtype="f64", product="f64", helm=so(4), pois=so(8))
    ws = (None if (args.no_learned or n < 6 or args.order != "interleaved")
          else W.WarmStart.load(ctx, Re, alpha, chi=16, bf16=True))
    mixed = F.step_opts(dt, tol=1e-8, chi=chi, dtype="f64", product=args.product, helm=so(4), pois=so(8), warm=ws)

    fields, sps, infos = {}, {}, {}
    paths = [("mixed", mixed)] + ([] if args.no_plain else [("plain", plain)])
    for name, opts in paths:
        print(f"[bench] {name} path", file=sys.stderr, flush=True)
        st, t, inf = run_path(Q, F, ctx, ops, U0, V0, P0, opts, args.warmup, args.steps, name)
        sps[name] = args.steps / t
        infos[name] = inf
        fields[name] = {k: dense(Q, F, getattr(st, k), n, args.order) for k in ("u", "v", "p")}
        if name == "mixed":
            st_m = st

    # roofline of the dominant kernel (the one-launch local CG) over one more step of the
    # mixed path; the step also hands out its pressure right-hand side b, so that the
    # global residual of its pressure solve can be read beside the projected one
    b_last = Q.MPS(L, chi)
    mixed_b = F.step_opts(dt, tol=1e-8, chi=chi, dtype="f64", product=args.product, helm=so(4), pois=so(8),
                          warm=ws, rhs_out=b_last)
    timer = Q.KernelTimer(ctx, "cg_coop", "f64")
    timer.start()
    info_last = F.fractional_step(ctx, ops, st_m, mixed_b)
    kt = timer.read()
    residual_last = None
    if not args.no_residual and int(max(ops.mpo["P"].bond_host)) * chi + b_last.cap > 512:
        residual_last = {"skipped": "w chi + chi exceeds the 512 capacity of qtt_add"}
    elif not args.no_residual:
        residual_last = {"projected": info_last.poisson.residual,
                         "global": global_residual(Q, ctx, ops.mpo["P"], st_m.p, b_last),
                         "step": "the step after the timed steps of the mixed path"}

    cpu, errs = None, None
    if not args.no_cpu:
        from oracle import diag
        g, ref, cpu = cpu_baseline(args, n, Re, dt, A0, u_init, v_init, args.warmup + args.steps)
        errs = {path: {k: float(diag.eps_l2(g, fl[k].ravel(), ref[k])) for k in ("u", "v", "p")}
                for path, fl in fields.items()}
    band = 3e-3
    in_band = {p: (errs is not None and max(e.values()) <= band) for p, e in (errs or {}).items()}
    reported = "mixed" if in_band.get("mixed", False) else ("plain" if "plain" in sps else "mixed")

    roof = None
    if kt["launches"] > 0 and kt["ms"] > 0:
        ach = kt["flops"] / (kt["ms"] * 1e-3) / 1e12
        prof = measured_profile()
        roof = {"bound": "mfma", "achieved": round(ach, 4), "peak": PEAKS["f64"], "unit": "TFLOP/s",
                "frac": round(ach / PEAKS["f64"], 6), "traffic": None if prof is None else round(prof["traffic"], 1),
                "kernel": "k_cg_coop (a site's whole local CG in one cooperative launch: both FP64 MFMA products "
                          "of every iteration, vector updates, barriers)",
                "avg_launch_us": round(1e3 * kt["ms"] / kt["launches"], 3), "launches": kt["launches"],
                "timing": "HIP-event bracket per launch on the library's stream",
                "idle_bracket_us": round(1e3 * kt["idle_bracket_ms"], 3),
                "kernel_trace_avg_us": None if prof is None else prof["trace_avg_us"],
                "flops_per_launch": round(kt["flops"] / kt["launches"], 1),
                "bytes_per_launch": round(kt["bytes"] / kt["launches"], 1)}

    def solver_summary(inf):
        return {"poisson_sweeps_mean": round(float(np.mean([i.poisson.sweeps for i in inf])), 3),
                "poisson_cg_iters_mean": round(float(np.mean([i.poisson.local_iters for i in inf])), 1),
                "poisson_residual_last": inf[-1].poisson.residual,
                "helmholtz_cg_iters_mean": round(float(np.mean([i.helm_u.local_iters for i in inf])), 1),
                "learned_guess_used": int(sum(i.warm_used for i in inf))}

    out = {
        "metric": "QTT fractional steps/s at 2^20 grid, chi=64: mixed+warm-start vs FP64, same error",
        "value": round(sps[reported], 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 / sps[reported], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if reported == "plain" else f"f64+{args.product}",
        "data": "synthetic",
        "config": {"workload": f"cylinder O-grid 2^{n}x2^{n} ({L} {args.order} cores), chi={chi}, Re={Re:g}, "
                               f"dt={dt:g}, App. G perturbation A0={A0:g}",
                   "reported_path": reported,
                   "mixed_path": f"FP64 fits (gradients, right-hand sides, divergence, projection), "
                                 f"{args.product.upper()}-MFMA Hadamard products, FP64 truncation, solves and "
                                 f"residuals, {'learned warm start' if ws else 'previous pressure'} of the pressure solve",
                   "plain_path": "FP64 throughout, previous pressure as the start of the pressure solve",
                   "solver_tol": args.tol, "local_tol": args.local_tol,
                   "mixed_steps_per_s": round(sps["mixed"], 4),
                   "plain_steps_per_s": None if "plain" not in sps else round(sps["plain"], 4),
                   "speedup_mixed_vs_plain": None if "plain" not in sps else round(sps["mixed"] / sps["plain"], 4),
                   "eps_l2_vs_oracle": errs, "within_3e-3": in_band,
                   "solver": {k: solver_summary(v) for k, v in infos.items()},
                   "poisson_residual_one_step": residual_last,
                   "setup_s": round(setup_s, 2)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
