"""Compression floor of the steady Re 40 record (results/c2_steady_re40_chi_sweep.json): the FD
oracle run over the same 2000 steps from the same initial field, then the error of the
best bond-chi approximation of its final u, v, p (TT-SVD of the dense fields in the
interleaved order), as the same |J|-weighted relative L2 error the record reports.
Calls the oracle only (test infrastructure); about a minute on one core. Writes
c2_best_approximation.txt beside this file.

    python tests/golden/c2_best_approximation.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from bench import initial_fields          # noqa: E402  (the record's initial-field recipe)
from oracle import diag, fd, qttref as R  # noqa: E402
from oracle.grid import OGrid             # noqa: E402


def main():
    n, Re, dt, steps = 8, 40.0, 5e-3, 2000
    g = OGrid(n, n)
    S = fd.FDSolver(g, Re, dt, solver="fft")
    u0, v0 = initial_fields(n, 1e-2)
    u, v = u0.ravel().copy(), v0.ravel().copy()
    for _ in range(steps):
        ref = S.step(u, v, return_stages=True)
        u, v = ref["u"], ref["v"]
    perm = R.grid_perm(n, n, "interleaved")
    lines = ["# chi, then the |J|-weighted relative L2 error of the best bond-chi approximation of the",
             "# FD oracle's u, v, p after 2000 steps (Re 40, 2^8 x 2^8, dt 5e-3, App. G modulation A0 1e-2)"]
    for chi in (16, 24, 32, 48, 64):
        err = {}
        for k in ("u", "v", "p"):
            f = ref[k]
            q = R.tt_full(R.tt_svd(f[perm], 2 * n, tol=0.0, chi_max=chi))
            grid = np.empty(4 ** n)
            grid[perm] = q
            err[k] = diag.eps_l2(g, grid, f)
        lines.append(f"{chi} " + " ".join(f"{err[k]:.3e}" for k in ("u", "v", "p")))
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "c2_best_approximation.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
