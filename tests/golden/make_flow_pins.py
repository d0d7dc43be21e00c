"""Writes the drag/lift histories of the dense FD oracle on the paper's cylinder cases.

Test infrastructure: calls only `oracle/`. Each case is the classical FD fractional
step (Sec. 3.3, App. A, App. E) run from the initial data the paper states for it;
drag and lift (App. F) are recorded every 10 steps into
tests/golden/<case>_forces.txt as rows (step, C_D, C_L). The tests compare the
printed FD values of the paper with these histories and re-run the first steps of
each case to check that the stored history is what the current oracle computes.

Cases (outer boundary at 32 D, i.e. r_out = 16, as in Sec. 4, except c3):
  rotating_g1_re100  G1 (2^8 x 2^8), Re = 100, rotation rate 1 (Eq. rot_bc), dt = 2e-3,
                     uniform start, 30000 steps (t = 60)          -> Table 2
  shedding_g2_re200  G2 (2^8 radial x 2^9 azimuthal), Re = 200, dt = 3.1e-3, uniform
                     start plus the App. G modulation with A0 = 0.05, 32258 steps (t = 100)
                                                                  -> Sec. 4.1.2, St ~ 0.1916
  steady_g2_re20     G2, Re = 20, dt = 3.8e-3, uniform start, 8100 steps -> Sec. 4.1.1
  c3_re200           2^10 x 2^10, r_out = 20, Re = 200, dt = 2e-3, A0 = 1e-2, 20000 steps
                     (t = 40): the reference of the TT path's long transient run

Usage: python tests/golden/make_flow_pins.py CASE [STEPS] [OUTDIR]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import diag, fd            # noqa: E402
from oracle.grid import OGrid           # noqa: E402

CASES = {
    "rotating_g1_re100": dict(n_eta=8, n_xi=8, r_out=16.0, Re=100.0, alpha=1.0, dt=2e-3, A0=0.0, steps=30000),
    "shedding_g2_re200": dict(n_eta=8, n_xi=9, r_out=16.0, Re=200.0, alpha=0.0, dt=3.1e-3, A0=0.05, steps=32258),
    "steady_g2_re20": dict(n_eta=8, n_xi=9, r_out=16.0, Re=20.0, alpha=0.0, dt=3.8e-3, A0=0.0, steps=8100),
    "c3_re200": dict(n_eta=10, n_xi=10, r_out=20.0, Re=200.0, alpha=0.0, dt=2e-3, A0=1e-2, steps=20000),
}
EVERY = 10


def run(case, steps=None, progress=None):
    """Yields (step, C_D, C_L) every EVERY steps of the FD run of `case`."""
    c = CASES[case]
    g = OGrid(c["n_eta"], c["n_xi"], r_out=c["r_out"])
    solver = fd.FDSolver(g, c["Re"], c["dt"], alpha=c["alpha"], solver="fft")
    u, v = fd.uniform_flow(g)
    if c["A0"]:
        u = u + fd.perturbation(g, c["A0"])
    bc = fd.velocity_bc(g, c["alpha"])
    for s in range(1, (steps or c["steps"]) + 1):
        st = solver.step(u, v, return_stages=True)
        u, v = st["u"], st["v"]
        if s % EVERY == 0:
            cd, cl = diag.forces(g, u, v, st["p"], c["Re"], bc["u_wall"], bc["v_wall"])
            if progress:
                progress(s, cd, cl)
            yield s, cd, cl


def path(case, outdir=HERE):
    return os.path.join(outdir, f"{case}_forces.txt")


def load(case, outdir=HERE):
    return np.loadtxt(path(case, outdir))


def main(case, steps=None, outdir=HERE):
    c = CASES[case]
    n = steps or c["steps"]
    t0 = time.time()
    rows = []

    def prog(s, cd, cl):
        if s % 1000 == 0:
            print(f"{case} step {s}/{n} t {s * c['dt']:.2f} C_D {cd:.5f} C_L {cl:.4e} {time.time() - t0:.0f} s",
                  flush=True)

    for r in run(case, n, prog):
        rows.append(r)
    hdr = (f"FD oracle drag/lift history, case {case}: " +
           ", ".join(f"{k}={v}" for k, v in c.items() if k != "steps") + f", steps={n}\n"
           f"written by: python tests/golden/make_flow_pins.py {case}\ncolumns: step C_D C_L (every {EVERY} steps)")
    np.savetxt(path(case, outdir), np.array(rows), fmt=["%d", "%.10e", "%.10e"], header=hdr)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 and sys.argv[2] else None,
         sys.argv[3] if len(sys.argv) > 3 else HERE)
