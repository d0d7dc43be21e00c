"""What the trained warm-start network gains, by a statistic stated before the run:
on the held-out cylinder configurations of the training run (Re and rotation rate
never seen in training) at 2^10 x 2^10, chi = 64, the median over configurations
of (local CG iterations of the pressure solve from a cold start) / (the same from
the learned start) is above 1, both solved to 1e-8 (or stopped at the same
sweep cap). The solver's reductions run in a fixed order, so the counts repeat.
The production start of a running simulation, the previous pressure, is reported
beside them (the learned guess is only taken when the solve's energy rates it
lower than the alternative)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_learned_start_median_gain_over_cold_start():
    from paper_2507_05222_amd import qtt as Q, warmstart as W
    with open(os.path.join(W.DATA, "wsnet.json")) as f:
        meta = json.load(f)
    ctx = Q.Context(0)
    gains, like = [], None
    for re, alpha in meta["test_configs"][:6]:
        r, like = W.compare_starts(ctx, re, alpha, like=like)
        cold, learned, prev = r["cold"], r["learned"], r["previous"]
        gains.append(cold["cg_iters"] / learned["cg_iters"])
        print(f"Re {re:.1f} alpha {alpha:.2f}: CG iterations cold {cold['cg_iters']} ({cold['sweeps']} sweeps), "
              f"learned {learned['cg_iters']} ({learned['sweeps']} sweeps, used {learned['warm_used']}), "
              f"previous pressure {prev['cg_iters']} ({prev['sweeps']} sweeps)", flush=True)
    assert float(np.median(gains)) > 1.0, gains
