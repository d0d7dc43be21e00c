"""Learned warm start of the pressure solve (binding): network parameters on the
GPU, training through the library's qtt_ws_* kernels (forward, squared error,
backward, Adam), the block-averaged 64 x 64 view of a train, and the model the
fractional step uses. Marshalling only; the arithmetic runs in libqtt.so."""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np
import torch

from . import qtt as Q

NPARAMS = 19681
CHANNELS = [(3, 32), (32, 32), (32, 32), (32, 1)]
HW = 64 * 64
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def init_params(seed=0) -> np.ndarray:
    """Glorot-uniform weights (limit sqrt(6 / (fan_in + fan_out)) over 3x3 taps), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in CHANNELS:
        lim = np.sqrt(6.0 / (9 * ci + 9 * co))
        parts.append(rng.uniform(-lim, lim, co * ci * 9))
        parts.append(np.zeros(co))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == NPARAMS
    return p


def coarse(ctx: Q.Context, m: Q.MPS) -> np.ndarray:
    """64 x 64 block average of a train in interleaved order (qtt_ws_coarse)."""
    g = np.empty(HW)
    ctx.check(Q.lib().qtt_ws_coarse(ctx.h, ctypes.byref(m.desc()), g.ctypes.data, Q._stream()))
    return g.reshape(64, 64)


def ws_input(b: np.ndarray, re: float, alpha: float):
    """Network input (3, 64, 64) of one block-averaged right-hand side and its scale
    rms(b) (qtt_ws_input_host, the rule the fractional step applies)."""
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(HW)
    x = np.empty(3 * HW, dtype=np.float32)
    r = ctypes.c_double(0)
    rc = Q.lib().qtt_ws_input_host(b.ctypes.data, float(re), float(alpha), x.ctypes.data, ctypes.byref(r))
    if rc != 0:
        raise Q.QttError(rc, "qtt_ws_input_host")
    return x.reshape(3, 64, 64), r.value


def _p(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Net:
    """The four-layer network with its Adam state (FP32, on the GPU)."""

    def __init__(self, ctx: Q.Context, params=None, seed=0):
        self.ctx = ctx
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        if p.size != NPARAMS:
            raise ValueError(f"expected {NPARAMS} parameters")
        self.params = torch.from_numpy(p.copy()).cuda()
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.steps = 0

    def forward(self, x: torch.Tensor, bf16=False):
        """x: [B][3][64][64] float32 on the GPU -> (out [B][1][64][64], activations)."""
        B = x.shape[0]
        x = x.contiguous()
        acts = torch.empty(Q.lib().qtt_ws_act_floats(B), dtype=torch.float32, device=x.device)
        out = torch.empty((B, 1, 64, 64), dtype=torch.float32, device=x.device)
        self.ctx.check(Q.lib().qtt_ws_forward(self.ctx.h, _p(self.params), _p(x), B, _p(acts), _p(out), int(bool(bf16)),
                                              Q._stream()))
        return out, acts

    def loss_grad(self, x: torch.Tensor, target: torch.Tensor):
        """Mean squared error and its gradient into self.grads (FP32 forward)."""
        B = x.shape[0]
        out, acts = self.forward(x)
        gout = torch.empty_like(out)
        part = torch.empty(64, dtype=torch.float32, device=x.device)
        n = out.numel()
        self.ctx.check(Q.lib().qtt_ws_mse(self.ctx.h, _p(out), _p(target.contiguous()), n, _p(gout), _p(part),
                                          Q._stream()))
        scratch = torch.empty(2 * B * 32 * HW, dtype=torch.float32, device=x.device)
        self.ctx.check(Q.lib().qtt_ws_backward(self.ctx.h, _p(self.params), _p(x.contiguous()), B, _p(acts), _p(gout),
                                               _p(self.grads), _p(scratch), Q._stream()))
        return float(part.sum().item()) / n

    def adam(self, lr: float):
        self.steps += 1
        self.ctx.check(Q.lib().qtt_ws_adam_step(self.ctx.h, _p(self.params), _p(self.grads), _p(self.m), _p(self.v),
                                                self.steps, ctypes.c_float(lr), Q._stream()))

    def numpy_params(self) -> np.ndarray:
        return self.params.detach().cpu().numpy().copy()


class WarmStart:
    """A trained network plus the constants the fractional step needs."""

    def __init__(self, ctx: Q.Context, params, out_scale, re, alpha=0.0, chi=16, bf16=True):
        self.net = Net(ctx, params)
        self.out_scale, self.re, self.alpha, self.chi, self.bf16 = float(out_scale), float(re), float(alpha), int(chi), bool(bf16)

    @classmethod
    def load(cls, ctx: Q.Context, re, alpha=0.0, chi=16, bf16=True, path=None):
        path = path or os.path.join(DATA, "wsnet.json")
        with open(path) as f:
            meta = json.load(f)
        params = np.load(os.path.join(os.path.dirname(path), meta["params"]), allow_pickle=False)
        return cls(ctx, params, meta["out_scale"], re, alpha, chi, bf16)

    def model(self) -> Q.CWsModel:
        return Q.CWsModel(self.net.params.data_ptr(), self.out_scale, self.re, self.alpha, self.chi, int(self.bf16))


def save(path_json: str, params: np.ndarray, out_scale: float, extra: dict | None = None):
    base = os.path.splitext(os.path.basename(path_json))[0]
    np.save(os.path.join(os.path.dirname(path_json), base + ".npy"), params.astype(np.float32), allow_pickle=False)
    meta = {"params": base + ".npy", "out_scale": float(out_scale), "n_params": NPARAMS}
    meta.update(extra or {})
    with open(path_json, "w") as f:
        json.dump(meta, f, indent=1)


def compare_starts(ctx: Q.Context, re: float, alpha: float, n=10, chi=64, dt=2e-3, history=24, tol=1e-8,
                   ws: "WarmStart | None" = None, like=None):
    """One fractional step of a flow `history` steps past uniform flow plus the App. G
    perturbation, its pressure solved to `tol` from three starts: "cold" (a seeded
    random train, no previous pressure), "learned" (the network's guess, rated by
    the solve's energy against that random train) and "previous" (the previous
    step's pressure, the start of a running simulation). Returns, per start, the
    step time, the pressure sweeps and CG iterations, the residual and whether the
    learned guess was taken. `like`: FlowOps of the same grid to share operators with."""
    import time
    from . import flow as F
    from qtt_inputs import random_mps_cores
    L = 2 * n
    N = 2 ** n
    i = np.arange(N)
    env = (np.exp((1.0 - (i + 1) / (N + 1)) ** 6) - 1.0) / (np.e - 1.0)
    u0 = 1.0 + 1e-2 * env[:, None] * np.sin(2 * np.pi * np.arange(N) / N)[None, :]
    ops = F.FlowOps(n, 20.0, re, dt, alpha, like=like)
    st = F.FlowState(Q.from_dense(ctx, F.grid_to_qtt_order(u0), L, 1e-14, chi, chi),
                     Q.from_dense(ctx, np.zeros(N * N), L, 1e-14, chi, chi),
                     Q.MPS.from_cores(random_mps_cores(L, chi, seed=0), chi))
    so = Q.solve_opts(tol=tol, max_sweeps=12, max_local_iters=80, local_tol=1e-2, dtype="f64")
    plain = F.step_opts(dt, tol=1e-8, chi=chi, dtype="f64", pois=so)
    for _ in range(history):
        F.fractional_step(ctx, ops, st, plain)
    ws = ws or WarmStart.load(ctx, re, alpha, chi=16, bf16=True)
    ws.re, ws.alpha = float(re), float(alpha)
    out = {}
    for name, warm, p0 in (("cold", None, None), ("learned", ws, None), ("previous", None, st.p)):
        p = Q.MPS(L, chi)
        p.copy_(p0 if p0 is not None else Q.MPS.from_cores(random_mps_cores(L, chi, seed=7), chi))
        s = F.FlowState(Q.MPS(L, chi).copy_(st.u), Q.MPS(L, chi).copy_(st.v), p)
        c2 = Q.Context(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = F.fractional_step(c2, ops, s, F.step_opts(dt, tol=1e-8, chi=chi, dtype="f64", pois=so, warm=warm))
        torch.cuda.synchronize()
        out[name] = {"step_s": time.perf_counter() - t0, "sweeps": info.poisson.sweeps,
                     "cg_iters": info.poisson.local_iters, "residual": info.poisson.residual,
                     "warm_used": int(info.warm_used)}
    return out, ops
