"""Host helpers of bench.py: the sweep's input canonicalisation and the exact MPO x MPS
product used by the global residual read-out, against the oracle's dense vectors."""
import numpy as np

from oracle import qttref as R
from qtt_inputs import random_mpo_cores, random_mps_cores


def test_left_canonical_keeps_the_vector_and_orthonormalises():
    import bench
    cores = random_mps_cores(10, 6, seed=5)
    lc = bench.left_canonical(cores)
    assert [c.shape for c in lc] == [c.shape for c in cores]
    for c in lc[:-1]:
        a, d, b = c.shape
        m = c.reshape(a * d, b)
        assert np.allclose(m.T @ m, np.eye(b), atol=1e-12)
    v, w = R.tt_full(cores), R.tt_full(lc)
    assert np.linalg.norm(v - w) <= 1e-12 * np.linalg.norm(v)


def test_exact_product_cores_match_the_dense_mpo_product():
    import bench
    x = random_mps_cores(8, 4, seed=6)
    M = random_mpo_cores(8, 3, seed=7)
    prod = bench.exact_product_cores(M, x)
    assert max(max(p.shape[0], p.shape[2]) for p in prod) <= 3 * 4
    ref = R.mpo_apply_dense(M, R.tt_full(x))
    assert np.linalg.norm(R.tt_full(prod) - ref) <= 1e-12 * np.linalg.norm(ref)
