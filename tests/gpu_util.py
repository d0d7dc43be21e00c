"""Helpers shared by the GPU tests (test code only)."""
import numpy as np


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def right_orthonormal_error(cores):
    """max over cores 1.. of ||C C^T - I|| with C = core reshaped (b_k, d b_{k+1})."""
    err = 0.0
    for c in cores[1:]:
        m = c.reshape(c.shape[0], -1)
        err = max(err, float(np.abs(m @ m.T - np.eye(m.shape[0])).max()))
    return err
