"""Drag and lift history of the transient cylinder (2^10 x 2^10 O-grid, Re = 200,
dt = 2e-3, uniform flow plus the App. G perturbation of amplitude 1e-2) from the
dense FP64 FD fractional step (Sec. 3.3, App. E), recorded every 10 steps.

Test infrastructure: the reference for the drag, lift, Strouhal number and lift
amplitude of the TT path's long run. Usage:

    python -m oracle.c3_force_history STEPS OUT.npy

OUT.npy holds rows (step, C_D, C_L) and is rewritten every 500 steps, so a long
run can be read while it goes.
"""
import sys
import time

import numpy as np

from oracle import diag, fd
from oracle.grid import OGrid

N_CORES, RE, DT, A0 = 10, 200.0, 2e-3, 1e-2


def main(steps, out):
    g = OGrid(N_CORES, N_CORES)
    solver = fd.FDSolver(g, RE, DT, solver="fft")
    u, v = fd.uniform_flow(g)
    u = u + fd.perturbation(g, A0)
    wall = fd.velocity_bc(g, 0.0)
    rows = []
    t0 = time.time()
    for s in range(1, steps + 1):
        st = solver.step(u, v, return_stages=True)
        u, v = st["u"], st["v"]
        if s % 10 == 0:
            cd, cl = diag.forces(g, u, v, st["p"], RE, wall["u_wall"], wall["v_wall"])
            rows.append((s, cd, cl))
        if s % 500 == 0 or s == steps:
            np.save(out, np.array(rows))
            print(f"step {s} t {s * DT:.2f} C_D {rows[-1][1]:.5f} C_L {rows[-1][2]:.4e} "
                  f"{time.time() - t0:.0f} s", flush=True)
    st_, amp = diag.strouhal(DT * np.array(rows)[:, 0], np.array(rows)[:, 2], min_periods=2)
    print(f"St {st_} lift amplitude {amp:.5f}", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]), sys.argv[2])
