"""Flow-level helpers of the binding: build the cylinder operators with the
library's host builder (or its TT-format builder), hold the GPU state (u, v, p) and call the fractional step.
Marshalling only; all arithmetic runs in libqtt.so."""
from __future__ import annotations

import ctypes
import itertools

import numpy as np

from . import qtt as Q


class FlowOps:
    """Operators (MPOs) and boundary vectors of a 2^n x 2^n O-grid (Sec. 3.2.3)."""

    # operators that depend on the grid only (not on Re, dt, the wall rotation or u_inf)
    GRID_ONLY = ("DX", "DZ", "DXP", "DZP", "WX", "WZ", "P", "JH", "JMH")

    def __init__(self, n, r_out=20.0, Re=100.0, dt=1e-3, alpha=0.0, u_inf=1.0, device="cuda", order="interleaved",
                 like=None, construction="host", ctx=None):
        """like: an FlowOps of the same grid (n, r_out, order) whose grid-only operators
        are shared instead of rebuilt; the Helmholtz operator and the boundary vectors
        are built for (Re, dt, alpha, u_inf).
        construction: "host" (every operator from qtt_build_host) or "tt" (the first
        derivatives, their pressure and |J|-weighted forms and the pressure operator built
        in TT format on the device by qtt_build_tt, Sec. 3.2.3; needs ctx)."""
        if construction not in ("host", "tt") or (construction == "tt" and ctx is None):
            raise ValueError("FlowOps: construction is 'host' or 'tt' (with ctx)")
        self.n, self.L = n, 2 * n
        self.order = order
        self.cyl = Q.cylinder(n, r_out, Re, dt, alpha, u_inf, order)
        names = ("DX", "DZ", "DXP", "DZP", "WX", "WZ", "HS", "P")
        if like is not None and (like.n, like.cyl.r_out, like.order) != (n, float(r_out), order):
            raise ValueError("FlowOps(like=...): a different grid")
        fresh = [k for k in names if like is None or k not in self.GRID_ONLY]
        built = {k: (self._tt(ctx, k) if construction == "tt" and k in Q.TT_OPS else Q.build_host(self.cyl, Q.OP[k]))
                 for k in fresh}
        # operators applied in one batched call share one slot capacity
        self.wcap = max([b[2] for b in built.values()] + ([like.wcap] if like is not None else []))
        if like is not None and self.wcap != like.wcap:
            raise ValueError("FlowOps(like=...): the Helmholtz operator needs another slot capacity")
        self.mpo = {k: Q.MPO(_relayout(built[k][0], built[k][2], self.wcap, 4), built[k][1], self.wcap, device)
                    for k in fresh}
        for k in names:
            if k not in self.mpo:
                self.mpo[k] = like.mpo[k]
        for k in ("JH", "JMH"):
            self.mpo[k] = like.mpo[k] if like is not None else Q.build_mpo(self.cyl, Q.OP[k], device)
        vnames = ("BX_U", "BZ_U", "BX_V", "BZ_V", "BL_U", "BL_V", "BW")
        bv = {k: Q.build_host(self.cyl, Q.VEC[k]) for k in vnames}
        self.bc_cap = max(b[2] for b in bv.values())
        self.vec = {k: Q.MPS.from_slots(_relayout(bv[k][0], bv[k][2], self.bc_cap, 2), bv[k][1], self.bc_cap, device)
                    for k in vnames}
        m, v = self.mpo, self.vec
        self.c = Q.CFlowOps(m["DX"].desc(), m["DZ"].desc(), m["DXP"].desc(), m["DZP"].desc(), m["WX"].desc(),
                            m["WZ"].desc(), m["HS"].desc(), m["P"].desc(), m["JH"].desc(), m["JMH"].desc(),
                            v["BX_U"].desc(), v["BZ_U"].desc(), v["BX_V"].desc(), v["BZ_V"].desc(),
                            v["BL_U"].desc(), v["BL_V"].desc(), v["BW"].desc())

    def _tt(self, ctx, k):
        m = Q.build_tt(ctx, self.cyl, Q.OP[k])
        return m.data.cpu().numpy(), m.bond_host.copy(), m.wcap

    def bonds(self):
        return {k: int(max(m.bond_host)) for k, m in self.mpo.items()}


def _relayout(slots, cap, cap_to, d):
    """Slots of a train (L cores of cap x d x cap) copied into slots of cap_to >= cap."""
    if cap == cap_to:
        return slots
    L = slots.size // (cap * d * cap)
    out = np.zeros((L, cap_to, d, cap_to))
    out[:, :cap, :, :cap] = slots.reshape(L, cap, d, cap)
    return out.reshape(-1)


class FlowState:
    """u, v, p of one flow. Each instance gets its own nonzero id: the library keys
    the warm start of a step's fits on it, not on storage addresses, which the
    allocator hands on to later states."""
    _ids = itertools.count(1)

    def __init__(self, u: Q.MPS, v: Q.MPS, p: Q.MPS):
        self.u, self.v, self.p = u, v, p
        self.id = next(FlowState._ids)

    def c(self):
        return Q.CFlowState(self.u.desc(), self.v.desc(), self.p.desc(), self.id)


def step_opts(dt, tol=1e-8, chi=64, dtype="f64", helm=None, pois=None, fit=2, product=None, warm=None,
              rhs_out=None) -> Q.CStepOpts:
    """dtype: contraction type of the fits (derivatives, right-hand sides, divergence,
    projection); product: that of the Hadamard (convection) products, default dtype.
    helm / pois: solver options (default: FP64 local products, tight tolerances).
    warm: a warmstart.WarmStart (learned initial guess of the pressure solve);
    rhs_out: an MPS that receives the pressure right-hand side."""
    prod = product or dtype
    helm = helm or Q.solve_opts(tol=1e-10, max_sweeps=4, max_local_iters=80, local_tol=1e-2, dtype="f64")
    pois = pois or Q.solve_opts(tol=1e-8, max_sweeps=8, max_local_iters=80, local_tol=1e-2, dtype="f64")
    o = Q.CStepOpts(float(dt), Q.CTrunc(float(tol), int(chi), int(fit)), Q.DTYPES.get(dtype, dtype),
                    Q.DTYPES.get(prod, prod), helm, pois)
    if warm is not None:
        o._warm = warm.model()            # keep the struct alive with the options
        o.warm = ctypes.pointer(o._warm)
    if rhs_out is not None:
        o._rhs = rhs_out.desc()
        o.rhs_out = ctypes.pointer(o._rhs)
    return o


def fractional_step(ctx: Q.Context, ops: FlowOps, st: FlowState, opts: Q.CStepOpts, stream=None):
    cs = st.c()
    info = Q.CStepInfo()
    ctx.check(Q.lib().qtt_fractional_step(ctx.h, ctypes.byref(ops.c), ctypes.byref(cs), ctypes.byref(opts),
                                          ctypes.byref(info), Q._stream(stream)))
    return info


def grid_to_qtt_order(field: np.ndarray, order="interleaved") -> np.ndarray:
    """(2^n, 2^n) grid array -> dense vector in the library's MSB-first bit order:
    interleaved (i_1 j_1 i_2 j_2 ...) or concatenated (i_1 .. i_n j_1 .. j_n)."""
    N = field.shape[0]
    n = int(np.log2(N))
    if order == "concatenated":
        return np.ascontiguousarray(field, dtype=np.float64).ravel().copy()
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    q = np.zeros_like(i)
    for m in range(n):
        q = (q << 2) | (((i >> (n - 1 - m)) & 1) << 1) | ((j >> (n - 1 - m)) & 1)
    out = np.empty(N * N)
    out[q.ravel()] = field.ravel()
    return out
