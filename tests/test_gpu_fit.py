"""GPU parity of the variational fit y ~ sum_t c_t M_t x_t against dense results."""
import numpy as np
import pytest

from oracle import qttref as R
from oracle.grid import OGrid
from qtt_inputs import random_mpo_cores, random_mps_cores
from tests.gpu_util import rel, right_orthonormal_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    from paper_2507_05222_amd import qtt
    return qtt


@pytest.fixture(scope="module")
def ctx(Q):
    return Q.Context(0)


def test_fit_sum_exact_full_rank(Q, ctx):
    """Full-rank bonds: the fit reproduces 0.7 M x - 1.3 z exactly (random start)."""
    L = 8
    M = random_mpo_cores(L, 3, seed=1)
    xc, zc = random_mps_cores(L, 4, seed=2), random_mps_cores(L, 5, seed=3)
    y = Q.MPS(L, 16)
    Q.fit(ctx, [[(0.7, Q.MPO.from_cores(M), Q.MPS.from_cores(xc, 4)), (-1.3, None, Q.MPS.from_cores(zc, 5))]], [y],
          chi=16, sweeps=2, init=1)
    ref = 0.7 * R.mpo_apply_dense(M, R.tt_full(xc)) - 1.3 * R.tt_full(zc)
    assert rel(R.tt_full(y.cores()), ref) < 1e-10
    assert right_orthonormal_error(y.cores()) < 1e-10


@pytest.mark.parametrize("dtype,bound", [("f32", 1e-5), ("bf16", 3e-2)])
def test_fit_low_precision(Q, ctx, dtype, bound):
    L = 8
    M = random_mpo_cores(L, 3, seed=4)
    xc = random_mps_cores(L, 4, seed=5)
    y = Q.MPS(L, 16)
    Q.fit(ctx, [[(1.0, Q.MPO.from_cores(M), Q.MPS.from_cores(xc, 4))]], [y], chi=16, sweeps=2, init=1, dtype=dtype)
    ref = R.mpo_apply_dense(M, R.tt_full(xc))
    assert rel(R.tt_full(y.cores()), ref) < bound
    assert right_orthonormal_error(y.cores()) < 1e-10


def _smooth(n):
    g = OGrid(n, n)
    X, Z = g.x_ext[2:-2], g.z_ext[2:-2]
    f = np.exp(-0.05 * (X ** 2 + Z ** 2)) * np.sin(0.7 * X) + 0.3 * np.cos(0.4 * Z)
    return f.ravel()[R.grid_perm(n, n)]


@pytest.mark.parametrize("chi", [8, 16])
def test_fit_truncated_quasi_optimal(Q, ctx, chi):
    """Curvilinear d/dx of a smooth field plus a boundary-like vector, truncated to chi:
    within 1.5x of the TT-SVD error of the exact result."""
    n = 6
    L = 2 * n
    x = Q.tt_svd_host(_smooth(n), L, 1e-12, 64, 64)
    D = Q.build_mpo(Q.cylinder(n), Q.OP["DX"])
    b = Q.build_vec(Q.cylinder(n), Q.VEC["BX_U"], 8)
    y = Q.MPS(L, 64)
    Q.fit(ctx, [[(1.0, D, x), (1.0, None, b)]], [y], chi=chi, sweeps=3, init=1)
    ref = R.mpo_apply_dense(D.cores(), R.tt_full(x.cores())) + R.tt_full(b.cores())
    err = rel(R.tt_full(y.cores()), ref)
    opt = rel(R.tt_full(R.tt_svd(ref, L, chi_max=chi)), ref)
    assert err <= 1.5 * opt + 1e-12, (err, opt)
    assert max(y.bonds()) <= chi


def test_fit_random_flat_spectrum(Q, ctx):
    """Random MPS and MPO (flat singular spectra, the hard case): within 1.5x of TT-SVD."""
    L, chi = 12, 16
    M = random_mpo_cores(L, 4, seed=6)
    xc = random_mps_cores(L, 16, seed=7)
    y = Q.MPS(L, chi)
    Q.fit(ctx, [[(1.0, Q.MPO.from_cores(M), Q.MPS.from_cores(xc, 16))]], [y], chi=chi, sweeps=4, init=1)
    ref = R.mpo_apply_dense(M, R.tt_full(xc))
    err = rel(R.tt_full(y.cores()), ref)
    opt = rel(R.tt_full(R.tt_svd(ref, L, chi_max=chi)), ref)
    assert err <= 1.5 * opt, (err, opt)


def test_fit_warm_start_and_batch(Q, ctx):
    """Two problems in one call; a warm restart from the result does not move it."""
    L = 8
    Ms = [random_mpo_cores(L, 2, seed=10 + i) for i in range(2)]
    xs = [random_mps_cores(L, 4, seed=20 + i) for i in range(2)]
    ys = [Q.MPS(L, 16) for _ in range(2)]
    probs = [[(1.0, Q.MPO.from_cores(Ms[i]), Q.MPS.from_cores(xs[i], 4))] for i in range(2)]
    Q.fit(ctx, probs, ys, chi=8, sweeps=2, init=1)
    first = [R.tt_full(y.cores()) for y in ys]
    Q.fit(ctx, probs, ys, chi=8, sweeps=1, init=0)
    for i in range(2):
        ref = R.mpo_apply_dense(Ms[i], R.tt_full(xs[i]))
        opt = rel(R.tt_full(R.tt_svd(ref, L, chi_max=8)), ref)
        assert rel(R.tt_full(ys[i].cores()), ref) <= 1.5 * opt + 1e-12
        assert rel(R.tt_full(ys[i].cores()), first[i]) < 1e-2


def test_fit_rank_deficient_target_stays_exact():
    """A rank-1 train fitted at bond 32 over 16 cores: the frame directions beyond the
    target's rank carry only rounding noise, which shrinks along the sweeps; the
    Householder moves must keep them finite (scale-invariant reflectors)."""
    import numpy as np
    from paper_2507_05222_amd import qtt as Q
    from oracle import qttref as R
    rng = np.random.default_rng(5)
    L, chi = 16, 32
    cores = [rng.standard_normal((1, 2, 1)) for _ in range(L)]
    x = Q.MPS.from_cores(cores, 2)
    ref = R.tt_full(cores)
    for sweeps in (1, 2, 3):
        y = Q.MPS(L, chi)
        Q.fit(Q.Context(0), [[(1.0, None, x)]], [y], chi=chi, sweeps=sweeps, init=1)
        got = R.tt_full(y.cores())
        assert np.isfinite(got).all(), sweeps
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref), sweeps
