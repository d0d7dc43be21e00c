"""CPU FP64 oracle for the QTT fractional-step method (arxiv 2507.05222).

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.

Contents (each function cites the passage of the paper it follows):
  grid    -- O-grid points (App. E, Eq. mesh) and metric terms (App. A).
  fd      -- the classical finite-difference twin of the scheme: curvilinear
             operators with ghost-point boundaries (Sec. 3.1, App. A), the
             Chorin fractional step (Sec. 3.3), sparse-LU and FFT/Thomas solves.
  qttref  -- dense-vector tensor-train reference: bit-order maps, TT-SVD,
             decompression, MPO action, inner products (Sec. 2, App. C/D).
  diag    -- diagnostics: weighted L2 error, forces, Strouhal number (Sec. 4, App. F).
  wsnet   -- FP64 forward/backward of the warm-start convolution network.

Parity status: every function here is pinned by a `-m "not gpu"` test against a
closed form, a printed value of the paper, or brute force, except where its
docstring says "parity unpinned".
"""
