"""GPU parity of the variational (ALS) solver against dense FP64 solves."""
import numpy as np
import pytest

from oracle import fd, qttref as R
from oracle.grid import OGrid
from qtt_inputs import random_mps_cores
from tests.gpu_util import rel, right_orthonormal_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    from paper_2507_05222_amd import qtt
    return qtt


@pytest.fixture(scope="module")
def ctx(Q):
    return Q.Context(0)


@pytest.mark.parametrize("which,Re,dt", [("P", 100.0, 1e-3), ("HS", 100.0, 1e-3)])
def test_als_full_rank_matches_dense(Q, ctx, which, Re, dt):
    """Full-rank bonds: the local problem spans the whole space, so ALS reaches the
    dense solution up to the CG tolerance."""
    n = 4
    L = 2 * n
    A = Q.build_mpo(Q.cylinder(n, Re=Re, dt=dt), Q.OP[which])
    Ad = R.mpo_full(A.cores())
    bc = random_mps_cores(L, 16, seed=3)
    x0 = random_mps_cores(L, 16, seed=4)
    b = Q.MPS.from_cores(bc, 16)
    x = Q.MPS.from_cores(x0, 16)
    opts = Q.solve_opts(tol=1e-9, max_sweeps=3, max_local_iters=400, local_tol=1e-12)
    info, ok = Q.poisson_solve(ctx, [A], [b], [x], opts)
    ref = np.linalg.solve(Ad, R.tt_full(bc))
    assert rel(R.tt_full(x.cores()), ref) < 1e-9, info[0].residual
    assert right_orthonormal_error(x.cores()) < 1e-10
    assert info[0].residual < 1e-7 and info[0].sweeps >= 1


def test_als_batched_two_rhs(Q, ctx):
    n = 4
    L = 2 * n
    A = Q.build_mpo(Q.cylinder(n, Re=50.0, dt=2e-3), Q.OP["HS"])
    Ad = R.mpo_full(A.cores())
    bs = [random_mps_cores(L, 16, seed=10 + i) for i in range(2)]
    B = [Q.MPS.from_cores(c, 16) for c in bs]
    X = [Q.MPS.from_cores(random_mps_cores(L, 16, seed=20 + i), 16) for i in range(2)]
    info, _ = Q.poisson_solve(ctx, [A, A], B, X, Q.solve_opts(tol=1e-10, max_sweeps=3, max_local_iters=200,
                                                                local_tol=1e-12))
    for i in range(2):
        assert rel(R.tt_full(X[i].cores()), np.linalg.solve(Ad, R.tt_full(bs[i]))) < 1e-9


def test_poisson_c1_grid_vs_fast_solver(Q, ctx):
    """The J-weighted pressure system on the 2^5 x 2^5 O-grid, full rank (chi_p = 32)."""
    n = 5
    L = 2 * n
    g = OGrid(n, n)
    P = Q.build_mpo(Q.cylinder(n), Q.OP["P"])
    rhs = np.random.default_rng(7).standard_normal(4 ** n)
    ref = fd.fast_poisson(g, rhs)                           # independent closed-form solver
    perm = R.grid_perm(n, n)
    b = Q.tt_svd_host(rhs[perm], L, 0.0, 32, 32)
    x = Q.MPS.from_cores(random_mps_cores(L, 32, seed=1), 32)
    info, _ = Q.poisson_solve(ctx, [P], [b], [x], Q.solve_opts(tol=1e-9, max_sweeps=2, max_local_iters=1500,
                                                               local_tol=1e-12))
    assert rel(R.tt_full(x.cores()), ref[perm]) < 1e-8, (info[0].residual, info[0].local_iters)


def test_als_capacity_64_full_rank_matches_dense(Q, ctx):
    """2^6 x 2^6 grid at slot capacity 64 (full rank): the local CG runs as one
    cooperative launch with four 32-row blocks per MPO index (the C3 shape)."""
    n = 6
    L = 2 * n
    A = Q.build_mpo(Q.cylinder(n, Re=100.0, dt=1e-3), Q.OP["P"])
    Ad = R.mpo_full(A.cores())
    bc = random_mps_cores(L, 64, seed=31)
    b = Q.MPS.from_cores(bc, 64)
    x = Q.MPS.from_cores(random_mps_cores(L, 64, seed=32), 64)
    opts = Q.solve_opts(tol=1e-10, max_sweeps=4, max_local_iters=600, local_tol=1e-12)
    info, _ = Q.poisson_solve(ctx, [A], [b], [x], opts)
    ref = np.linalg.solve(Ad, R.tt_full(bc))
    assert rel(R.tt_full(x.cores()), ref) < 1e-8, (info[0].residual, info[0].sweeps, info[0].local_iters)
    assert right_orthonormal_error(x.cores()) < 1e-10


def test_solve_is_bitwise_reproducible(Q, ctx):
    """The same truncated solve twice (fresh contexts): identical cores, residuals and
    iteration counts, since every reduction of the solver runs in a fixed order."""
    n = 5
    L = 2 * n
    A = Q.build_mpo(Q.cylinder(n, Re=100.0, dt=1e-3), Q.OP["P"])
    bc = random_mps_cores(L, 16, seed=33)
    runs = []
    for _ in range(2):
        c = Q.Context(0)
        b = Q.MPS.from_cores(bc, 16)
        x = Q.MPS.from_cores(random_mps_cores(L, 16, seed=34), 16)
        info, _ = Q.poisson_solve(c, [A], [b], [x], Q.solve_opts(tol=1e-12, max_sweeps=3, max_local_iters=80,
                                                                local_tol=1e-2))
        runs.append(([cc.copy() for cc in x.cores()], info[0].local_iters, info[0].residual))
    (xa, ia, ra), (xb, ib, rb) = runs
    assert ia == ib and ra == rb
    assert all(np.array_equal(p, q) for p, q in zip(xa, xb))


@pytest.mark.parametrize("chi_x,tol", [(4, 1e-3), (16, 1e-10)])
def test_global_residual_readout_matches_dense(Q, ctx, chi_x, tol):
    """The bench's global residual ||A x - b|| / ||b|| (exact product, rounded difference, norm)
    against the dense residual: a bond-limited solve (large residual) and a full-rank one
    (residual near round-off), where the expanded inner-product form would cancel."""
    import bench
    n = 4
    L = 2 * n
    A = Q.build_mpo(Q.cylinder(n, Re=100.0, dt=1e-3), Q.OP["P"])
    Ad = R.mpo_full(A.cores())
    bc = random_mps_cores(L, 16, seed=31)
    b = Q.MPS.from_cores(bc, 16)
    x = Q.MPS.from_cores(random_mps_cores(L, chi_x, seed=32), chi_x)
    Q.poisson_solve(ctx, [A], [b], [x], Q.solve_opts(tol=tol, max_sweeps=4, max_local_iters=400, local_tol=1e-12))
    bd = R.tt_full(bc)
    dense = np.linalg.norm(Ad @ R.tt_full(x.cores()) - bd) / np.linalg.norm(bd)
    g = bench.global_residual(Q, ctx, A, x, b)
    assert abs(g - dense) <= 1e-12 + 1e-6 * dense, (g, dense)
