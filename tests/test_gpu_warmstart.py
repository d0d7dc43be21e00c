"""What the trained warm-start network gains: on held-out cylinder configurations
(Re, rotation rate never seen in training) at 2^10 x 2^10, chi = 64, the pressure
solve of a step started from the network's prediction needs fewer local CG
iterations to the same tolerance (1e-8) than the same solve started cold (a
seeded random train)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run(re, alpha, n=10, chi=64, dt=2e-3, history=3):
    from paper_2507_05222_amd import flow as F, qtt as Q, warmstart as W
    from qtt_inputs import random_mps_cores
    import bench
    L = 2 * n
    ctx = Q.Context(0)
    ops = F.FlowOps(n, 20.0, re, dt, alpha)
    u0, v0 = bench.initial_fields(n, 1e-2)
    st = F.FlowState(Q.tt_svd_host(F.grid_to_qtt_order(u0), L, 1e-14, chi, chi),
                     Q.tt_svd_host(F.grid_to_qtt_order(v0), L, 1e-14, chi, chi),
                     Q.MPS.from_cores(random_mps_cores(L, chi, seed=0), chi))
    so = Q.solve_opts(tol=1e-8, max_sweeps=12, max_local_iters=80, local_tol=1e-2, dtype="f64")
    plain = F.step_opts(dt, tol=1e-8, chi=chi, dtype="f64", pois=so)
    for _ in range(history):
        F.fractional_step(ctx, ops, st, plain)
    ws = W.WarmStart.load(ctx, re, alpha, chi=16, bf16=True)
    out = {}
    for name, warm in (("cold", None), ("learned", ws)):
        s = F.FlowState(Q.MPS(L, chi).copy_(st.u), Q.MPS(L, chi).copy_(st.v),
                        Q.MPS.from_cores(random_mps_cores(L, chi, seed=7), chi))     # no previous pressure
        info = F.fractional_step(Q.Context(0), ops, s, F.step_opts(dt, tol=1e-8, chi=chi, dtype="f64", pois=so, warm=warm))
        out[name] = info
    return out


def test_learned_start_beats_cold_start():
    from paper_2507_05222_amd import warmstart as W
    with open(os.path.join(W.DATA, "wsnet.json")) as f:
        meta = json.load(f)
    gains = []
    for re, alpha in meta["test_configs"][:2]:
        r = _run(re, alpha)
        cold, learned = r["cold"], r["learned"]
        assert learned.warm_used == 1 and learned.warm_energy < learned.prev_energy
        assert learned.poisson.residual <= 1e-8 and cold.poisson.residual <= 1e-8
        gains.append(cold.poisson.local_iters / learned.poisson.local_iters)
        print(f"Re {re:.1f} alpha {alpha:.2f}: CG iterations cold {cold.poisson.local_iters} "
              f"({cold.poisson.sweeps} sweeps), learned {learned.poisson.local_iters} ({learned.poisson.sweeps} sweeps)")
    assert min(gains) > 1.0, gains
