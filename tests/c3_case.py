"""The 2^10 x 2^10 transient cylinder case (Re = 200, dt = 2e-3, chi = 64) run
through the HIP fractional step and through the FD oracle from the same initial
fields (uniform flow plus the App. G perturbation). Test infrastructure."""
import numpy as np

from oracle import diag, fd, qttref as R
from oracle.grid import OGrid
from qtt_inputs import random_mps_cores

N_CORES, CHI, RE, DT, A0, R_OUT = 10, 64, 200.0, 2e-3, 1e-2, 20.0


def solve_opts_for(dtype, tol=1e-9):
    from paper_2507_05222_amd import qtt as Q
    helm = Q.solve_opts(tol=tol, max_sweeps=4, max_local_iters=80, local_tol=1e-2, dtype=dtype)
    pois = Q.solve_opts(tol=tol, max_sweeps=8, max_local_iters=80, local_tol=1e-2, dtype=dtype)
    return helm, pois


def run(nsteps, n=N_CORES, chi=CHI, dtype="f64", product=None, return_state=False, solver_dtype=None,
        learned=False, tol=1e-9):
    """Per-step eps_L2 of (u, v, p) against the oracle and the solver infos (and, with
    return_state, the final TT state, the oracle's last stage dict, the context and ops).
    dtype: MFMA type of the fits; product: of the Hadamard products; solver_dtype: of the
    solves' local products (default dtype); learned: the learned warm start of the
    pressure solve; tol: the solves' residual tolerance."""
    from paper_2507_05222_amd import flow as F, qtt as Q
    L = 2 * n
    g = OGrid(n, n)
    u0, v0 = fd.uniform_flow(g)
    u0 = u0 + fd.perturbation(g, A0)
    perm = R.grid_perm(n, n)
    ctx = Q.Context(0)
    ops = F.FlowOps(n, R_OUT, RE, DT)
    st = F.FlowState(Q.tt_svd_host(u0[perm], L, 1e-14, chi, chi), Q.tt_svd_host(v0[perm] + 0.0, L, 1e-14, chi, chi),
                     Q.MPS.from_cores(random_mps_cores(L, chi, seed=0), chi))
    helm, pois = solve_opts_for(solver_dtype or dtype, tol)
    ws = None
    if learned:
        from paper_2507_05222_amd import warmstart as W
        ws = W.WarmStart.load(ctx, RE, 0.0, chi=16, bf16=True)
    opts = F.step_opts(DT, tol=1e-8, chi=chi, dtype=dtype, helm=helm, pois=pois, product=product, warm=ws)
    S = fd.FDSolver(g, RE, DT, solver="fft")
    u, v = u0.copy(), v0.copy()
    out = []
    for _ in range(nsteps):
        info = F.fractional_step(ctx, ops, st, opts)
        ref = S.step(u, v, return_stages=True)
        u, v = ref["u"], ref["v"]
        errs = {}
        for name, m in (("u", st.u), ("v", st.v), ("p", st.p)):
            grid = np.empty(4 ** n)
            grid[perm] = R.tt_full(m.cores())
            errs[name] = diag.eps_l2(g, grid, ref[name])
        out.append((errs, info))
    if return_state:
        return out, st, ref, ctx, ops
    return out
