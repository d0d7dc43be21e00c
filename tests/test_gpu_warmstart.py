"""What the trained warm-start network gains: on held-out cylinder configurations
(Re, rotation rate never seen in training) at 2^10 x 2^10, chi = 64, the pressure
solve of a step started from the network's prediction needs fewer local CG
iterations to the same tolerance (1e-8) than the same solve started cold (a
seeded random train)."""
import json
import os

import pytest

pytestmark = pytest.mark.gpu


def test_learned_start_beats_cold_start():
    from paper_2507_05222_amd import qtt as Q, warmstart as W
    with open(os.path.join(W.DATA, "wsnet.json")) as f:
        meta = json.load(f)
    gains = []
    for re, alpha in meta["test_configs"][:2]:
        r = W.compare_cold_learned(Q.Context(0), re, alpha)
        cold, learned = r["cold"], r["learned"]
        assert learned["warm_used"] == 1
        assert learned["residual"] <= 1e-8 and cold["residual"] <= 1e-8
        gains.append(cold["cg_iters"] / learned["cg_iters"])
        print(f"Re {re:.1f} alpha {alpha:.2f}: CG iterations cold {cold['cg_iters']} ({cold['sweeps']} sweeps), "
              f"learned {learned['cg_iters']} ({learned['sweeps']} sweeps)")
    assert min(gains) > 1.0, gains
