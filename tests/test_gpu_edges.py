"""GPU parity at the edges of the method's input space: the shortest chains and
bond-1 (product) trains, the zero train, the largest slot capacity the library
supports (256: the generic Householder kernels, the two-kernel zip-up and 512 x 512
Gram matrices), and the error returns of malformed calls."""
import numpy as np
import pytest

from oracle import qttref as R
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


def _rc(Q, ctx, cores, cap):
    x = Q.MPS.from_cores(cores, cap)
    Q.round_(ctx, [x], tol=0.0, chi=cap)
    return x


@pytest.mark.parametrize("L,chi,w", [(2, 2, 2), (2, 1, 1), (6, 1, 3)])
def test_short_and_product_trains(Q, ctx, L, chi, w):
    """L = 2 (one bond) and bond-1 trains: apply, round, add and dot against the
    dense oracle."""
    xc = random_mps_cores(L, chi, seed=60)
    yc = random_mps_cores(L, chi, seed=61)
    M = random_mpo_cores(L, w, seed=62)
    cap = max(chi * w, 2)
    x = _rc(Q, ctx, xc, cap)
    y = Q.MPS(L, cap)
    Q.apply_mpo(ctx, [Q.MPO.from_cores(M)], [x], [y], tol=0.0, chi=cap)
    assert rel(R.tt_full(y.cores()), R.mpo_apply_dense(M, R.tt_full(xc))) < 1e-12
    z = Q.MPS(L, 2 * cap)
    Q.add(ctx, 0.5, [x], -2.0, [Q.MPS.from_cores(yc, cap)], [z], tol=0.0, chi=2 * cap)
    assert rel(R.tt_full(z.cores()), 0.5 * R.tt_full(xc) - 2.0 * R.tt_full(yc)) < 1e-12
    d = Q.dot(ctx, [x], [Q.MPS.from_cores(yc, cap)])[0]
    assert abs(d - R.tt_full(xc) @ R.tt_full(yc)) < 1e-12 * np.linalg.norm(R.tt_full(xc)) * np.linalg.norm(R.tt_full(yc))


def test_zero_train(Q, ctx):
    """The zero vector through apply, round, add, dot, fit and solve: zero results,
    finite cores (no 0/0 in the factorisations), orthonormal gauges where promised."""
    L, chi = 8, 8
    zero = Q.MPS.from_cores([np.zeros((1 if k == 0 else chi, 2, 1 if k == L - 1 else chi)) for k in range(L)], chi)
    xc = random_mps_cores(L, chi, seed=63)
    x = _rc(Q, ctx, xc, chi)
    M = random_mpo_cores(L, 3, seed=64)
    y = Q.MPS(L, 3 * chi)
    Q.apply_mpo(ctx, [Q.MPO.from_cores(M)], [zero], [y], tol=0.0, chi=3 * chi)
    assert np.isfinite(np.concatenate([c.ravel() for c in y.cores()])).all()
    assert np.abs(R.tt_full(y.cores())).max() == 0.0
    r = Q.MPS(L, chi)
    r.copy_(zero)
    Q.round_(ctx, [r], tol=1e-8, chi=chi)
    assert np.isfinite(np.concatenate([c.ravel() for c in r.cores()])).all()
    assert np.abs(R.tt_full(r.cores())).max() == 0.0
    z = Q.MPS(L, 2 * chi)
    Q.add(ctx, 1.0, [x], -1.0, [x], [z], tol=1e-12, chi=2 * chi)
    assert np.linalg.norm(R.tt_full(z.cores())) <= 1e-13 * np.linalg.norm(R.tt_full(xc))
    assert Q.dot(ctx, [zero], [x])[0] == 0.0
    f = Q.MPS(L, chi)
    Q.fit(ctx, [[(1.0, None, zero)]], [f], chi=chi, sweeps=2, init=1)
    assert np.isfinite(np.concatenate([c.ravel() for c in f.cores()])).all()
    assert np.abs(R.tt_full(f.cores())).max() == 0.0
    # solve A x = 0 from a nonzero start: x = 0
    A = Q.build_mpo(Q.cylinder(4, Re=100.0, dt=1e-3), Q.OP["HS"])
    b0 = Q.MPS.from_cores([np.zeros((1 if k == 0 else 4, 2, 1 if k == 7 else 4)) for k in range(8)], 16)
    xs = Q.MPS.from_cores(random_mps_cores(8, 16, seed=65), 16)
    info, ok = Q.poisson_solve(ctx, [A], [b0], [xs], Q.solve_opts(tol=1e-10, max_sweeps=2))
    assert ok and info[0].residual == 0.0
    assert np.abs(R.tt_full(xs.cores())).max() == 0.0


def test_capacity_256_apply_exact(Q, ctx):
    """Slot capacity 256 (largest): input bond 128, MPO bond 2, L = 18, so the exact
    product has bonds up to 256 = the output capacity and the zip-up Gram matrices
    reach 512 x 512; the contraction runs as two kernels (capacity above 128)."""
    L = 18
    xc = random_mps_cores(L, 128, seed=66)
    M = random_mpo_cores(L, 2, seed=67)
    x = _rc(Q, ctx, xc, 256)
    y = Q.MPS(L, 256)
    Q.apply_mpo(ctx, [Q.MPO.from_cores(M)], [x], [y], tol=0.0, chi=256)
    assert max(y.bonds()) == 256
    assert rel(R.tt_full(y.cores()), R.mpo_apply_dense(M, R.tt_full(xc))) < 1e-10
    assert right_orthonormal_error(y.cores()) < 1e-10


def test_capacity_256_fit_and_solve(Q, ctx):
    """Capacity 256 selects the generic (LDS / global) Householder kernels in the fit
    and the solver: an exact fit of a bond-128 train, and a full-rank solve."""
    L = 16
    xc = random_mps_cores(L, 128, seed=68)
    x = Q.MPS.from_cores(xc, 256)
    f = Q.MPS(L, 256)
    Q.fit(ctx, [[(1.5, None, x)]], [f], chi=256, sweeps=2, init=1)
    assert rel(R.tt_full(f.cores()), 1.5 * R.tt_full(xc)) < 1e-10
    n = 4
    A = Q.build_mpo(Q.cylinder(n, Re=100.0, dt=1e-3), Q.OP["P"])
    bc = random_mps_cores(2 * n, 16, seed=69)
    b = Q.MPS.from_cores(bc, 256)
    xs = Q.MPS.from_cores(random_mps_cores(2 * n, 16, seed=70), 256)
    info, _ = Q.poisson_solve(ctx, [A], [b], [xs], Q.solve_opts(tol=1e-9, max_sweeps=3, max_local_iters=400,
                                                                local_tol=1e-12))
    ref = np.linalg.solve(R.mpo_full(A.cores()), R.tt_full(bc))
    assert rel(R.tt_full(xs.cores()), ref) < 1e-9
    assert right_orthonormal_error(xs.cores()) < 1e-10


def test_malformed_calls_return_errors(Q, ctx):
    """Shape and capacity errors come back as codes (no launch, no output written)."""
    x8 = Q.MPS.from_cores(random_mps_cores(8, 4, seed=71), 4)
    x6 = Q.MPS.from_cores(random_mps_cores(6, 4, seed=72), 4)
    M8 = Q.MPO.from_cores(random_mpo_cores(8, 2, seed=73))
    y6 = Q.MPS(6, 8)
    with pytest.raises(Q.QttError, match="ESHAPE"):
        Q.apply_mpo(ctx, [M8], [x6], [y6], tol=0.0, chi=8)
    with pytest.raises(Q.QttError, match="ECAPACITY"):
        Q.fit(ctx, [[(1.0, None, x8)]], [Q.MPS(8, 4)], chi=8, sweeps=1, init=1)
    with pytest.raises(Q.QttError):
        Q.dot(ctx, [x8], [x6])
    big = Q.MPS(8, 300)
    with pytest.raises(Q.QttError, match="ESHAPE"):
        Q.poisson_solve(ctx, [M8], [big], [Q.MPS(8, 300)], Q.solve_opts())
    # the zip-up factorises Gram matrices of order 2 * bond in one workgroup: an
    # output bond above 256 is refused before any launch
    y512 = Q.MPS(8, 512)
    with pytest.raises(Q.QttError, match="ESHAPE"):
        Q.apply_mpo(ctx, [M8], [x8], [y512], tol=0.0, chi=512)
