"""The oracle's assembled fractional step against the FD values the paper prints.

The force histories in tests/golden/<case>_forces.txt are written by
tests/golden/make_flow_pins.py, which calls only `oracle/` (the classical FD step of
Sec. 3.3 on the paper's grids and initial data). Two checks per case:

* the stored history is what the current oracle computes: its first rows are
  recomputed here and must agree to rounding;
* the history reproduces the FD numbers the paper prints for that case
  (tests/golden/paper_numbers.json, "fd_pins", each with its citation).

What this pins beyond the stencil and solver tests: the assembly of the step
(convection sign and terms, boundary-correction scales, the order of predictor,
pressure and projection), the rotating wall condition (Eq. rot_bc: its sign sets the
sign of the mean lift) and the force read-out (App. F). Tolerance 2%: the wall
pressure ghost value and the wall stress stencil are readings where the paper gives
no formula, and its grids' exact outer radius and time step are rounded in the text.
"""
import json
import os

import numpy as np
import pytest

from oracle import diag
from tests.golden import make_flow_pins as M

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "paper_numbers.json")) as f:
    PINS = {(p["case"], p["quantity"]): p for p in json.load(f)["fd_pins"]}
REL = 0.02


def _hist(case):
    h = M.load(case)
    assert h.ndim == 2 and h.shape[1] == 3
    return h


@pytest.mark.parametrize("case,steps", [("rotating_g1_re100", 200), ("shedding_g2_re200", 200),
                                        ("steady_g2_re20", 200),
                                        pytest.param("c3_re200", 20, marks=pytest.mark.skipif(
                                            not os.path.exists(M.path("c3_re200")), reason="C3 history not written"))])
def test_stored_history_is_the_oracles(case, steps):
    """The first rows of the stored history equal a fresh run of the oracle."""
    h = _hist(case)
    fresh = np.array(list(M.run(case, steps)))
    n = len(fresh)
    assert n == steps // M.EVERY and np.array_equal(h[:n, 0], fresh[:, 0])
    np.testing.assert_allclose(h[:n, 1:], fresh[:, 1:], rtol=1e-9, atol=1e-12)


def test_rotating_cylinder_table2():
    """Re = 100, rotation rate 1, G1: mean lift and lift Strouhal number over the last
    half of the run (t = 30 .. 60) against the FD row of Table 2."""
    h = _hist("rotating_g1_re100")
    dt = M.CASES["rotating_g1_re100"]["dt"]
    t, cl = h[:, 0] * dt, h[:, 2]
    half = t >= 0.5 * t[-1]
    cl_mean = float(cl[half].mean())
    St, _ = diag.strouhal(t, cl)
    ref_cl = PINS[("rotating_g1_re100", "mean_C_L")]["value"]
    ref_st = PINS[("rotating_g1_re100", "St")]["value"]
    assert cl_mean > 0.0                       # sign of Eq. rot_bc: lift towards +z
    assert abs(cl_mean - ref_cl) <= REL * ref_cl, cl_mean
    assert St is not None and abs(St - ref_st) <= REL * ref_st, St


def test_shedding_strouhal_re200_g2():
    """Re = 200, G2, App. G modulation (A0 = 0.05): Strouhal number from interpolated
    upward zero crossings of C_L over t = 50 .. 100 (Sec. 4.1.2). The paper prints
    the FD value as 0.1916 and calls it 1e-3 from the literature's 0.1977, numbers
    6.1e-3 apart; the pin is the range between them, widened by the same 2%."""
    h = _hist("shedding_g2_re200")
    dt = M.CASES["shedding_g2_re200"]["dt"]
    t = h[:, 0] * dt
    assert t[-1] >= 99.9
    St, amp = diag.strouhal(t, h[:, 2])
    pin = PINS[("shedding_g2_re200", "St")]
    lo, hi = (1.0 - REL) * pin["value"], (1.0 + REL) * pin["literature"]
    assert amp > 0.1                           # a developed Karman street
    assert St is not None and lo <= St <= hi, St
    # periodic: the two halves of the window give the same frequency
    half = t >= 75.0
    St2, _ = diag.strouhal(t[half], h[half, 2], window=1.0)
    assert abs(St2 - St) <= 1e-3 * St


def test_steady_re20_lift_negligible():
    """Re = 20, G2, 8100 steps from uniform flow: the lift stays at the FD level the
    paper reports (|C_L| ~ 1e-4), the flow being symmetric; the drag has settled."""
    h = _hist("steady_g2_re20")
    assert int(h[-1, 0]) == 8100
    ref = PINS[("steady_g2_re20", "abs_C_L_max")]["value"]
    assert abs(h[-1, 2]) <= ref
    # settled: the drag changes by less than 0.1% over the last 1000 steps
    last = h[h[:, 0] >= 7100, 1]
    assert abs(last[-1] - last[0]) <= 1e-3 * abs(last[-1])


@pytest.mark.skipif(not os.path.exists(M.path("c3_re200")), reason="C3 history not written")
def test_c3_history_complete():
    """The reference history of the 2^10 x 2^10 transient run covers t = 0 .. 40."""
    h = _hist("c3_re200")
    assert int(h[-1, 0]) == M.CASES["c3_re200"]["steps"]
    assert np.all(np.isfinite(h))
