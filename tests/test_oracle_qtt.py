"""Pins of the dense-vector TT reference (oracle/qttref.py) against the paper and closed forms."""
import json
import os

import numpy as np
import pytest

from oracle import qttref as q
from qtt_inputs import bond_profile, random_mps_cores

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_app_d_worked_example():
    """App. D: the three printed cores contract to t = (1..8); first core = most significant digit."""
    d = json.load(open(os.path.join(GOLD, "app_d_example.json")))
    cores = [np.array(c, dtype=float) for c in d["cores"]]
    np.testing.assert_array_equal(q.tt_full(cores), np.array(d["vector"], dtype=float))
    np.testing.assert_array_equal(q.tt_full(q.app_d_cores()), np.arange(1, 9, dtype=float))
    # reversing the digit significance (last core most significant) would give a different vector
    rev = [np.transpose(c, (2, 1, 0)) for c in cores[::-1]]
    assert not np.array_equal(q.tt_full(rev), np.arange(1, 9))


def test_qtt_index_brute_force():
    n = 3
    for i in range(8):
        for j in range(8):
            ib, jb = format(i, "03b"), format(j, "03b")
            inter = int("".join(a + b for a, b in zip(ib, jb)), 2)
            assert q.qtt_index(i, j, n, n, "interleaved") == inter
            assert q.qtt_index(i, j, n, n, "concatenated") == int(ib + jb, 2)
    f = np.arange(64.0).reshape(8, 8)
    np.testing.assert_array_equal(q.qtt_to_grid(q.grid_to_qtt(f), 3, 3), f)
    perm = q.grid_perm(3, 3)
    np.testing.assert_array_equal(f.ravel()[perm], q.grid_to_qtt(f))


def test_nvps_printed_percentages():
    d = json.load(open(os.path.join(GOLD, "paper_numbers.json")))
    for e in d["nvps_percent"]:
        pct = 100.0 * q.nvps(q.bond_cap_profile(e["L"], e["chi"])) / 2 ** e["L"]
        # the paper rounds its percentages; its most precise one is 5.8 (we get 5.77)
        assert abs(pct - e["percent"]) < 0.6 * max(1.0, e["percent"] / 10.0), (e, pct)
    m = d["max_chi_G1"]
    assert max(q.bond_cap_profile(m["L"], 10 ** 9)) == m["chi"]
    assert q.bond_cap_profile(10, 8) == bond_profile(10, 8)


@pytest.mark.parametrize("tol", [1e-1, 1e-3, 1e-6, 1e-10])
def test_tt_svd_error_bound(tol):
    rng = np.random.default_rng(3)
    # a vector with decaying spectrum at every unfolding
    v = q.tt_full(random_mps_cores(12, 16, seed=5)) + 1e-4 * rng.standard_normal(2 ** 12)
    cores = q.tt_svd(v, 12, tol=tol)
    err = np.linalg.norm(q.tt_full(cores) - v) / np.linalg.norm(v)
    assert err <= tol * (1 + 1e-10)
    prof = q.bond_cap_profile(12, 10 ** 9)
    assert all(b <= c for b, c in zip(q.bonds_of(cores), prof))


def test_tt_svd_exact_and_closed_form_ranks():
    rng = np.random.default_rng(0)
    v = rng.standard_normal(2 ** 10)
    cores = q.tt_svd(v, 10, tol=0.0)
    assert np.linalg.norm(q.tt_full(cores) - v) < 1e-12 * np.linalg.norm(v)
    j = np.arange(2 ** 12)
    # closed-form QTT ranks: exponential 1, sine 2, linear 2 (analytic TT constructions)
    for f, r in [(np.exp(0.01 * j), 1), (np.sin(2 * np.pi * j / 2 ** 12 * 3), 2), (1.0 + j, 2)]:
        b = q.bonds_of(q.tt_svd(f, 12, tol=1e-12))
        assert max(b) == r, (r, b)


def test_chi_cap_is_optimal_at_one_bond():
    """With one cut, TT-SVD capped at chi equals the Eckart-Young optimum."""
    rng = np.random.default_rng(1)
    M = rng.standard_normal((8, 8))
    v = M.reshape(-1)
    s = np.linalg.svd(M, compute_uv=False)
    cores = q.tt_svd(v, 2, d=8, tol=0.0, chi_max=3)
    err = np.linalg.norm(q.tt_full(cores) - v)
    assert abs(err - np.sqrt(np.sum(s[3:] ** 2))) < 1e-12


def test_mpo_action_kron_closed_form():
    """A bond-1 MPO is the Kronecker product of its 2x2 cores (first core most significant)."""
    rng = np.random.default_rng(2)
    cores = [rng.standard_normal((1, 2, 2, 1)) for _ in range(6)]
    K = np.array([[1.0]])
    for c in cores:
        K = np.kron(K, c[0, :, :, 0])
    np.testing.assert_allclose(q.mpo_full(cores), K, rtol=1e-13, atol=1e-13)
    x = rng.standard_normal(64)
    np.testing.assert_allclose(q.mpo_apply_dense(cores, x), K @ x, rtol=1e-12, atol=1e-12)


def test_mpo_apply_and_dots_vs_dense():
    rng = np.random.default_rng(4)
    L = 8
    mpo = [rng.standard_normal((1 if k == 0 else 3, 2, 2, 1 if k == L - 1 else 3)) for k in range(L)]
    x = random_mps_cores(L, 5, seed=1)
    y = random_mps_cores(L, 4, seed=2)
    X, Y, M = q.tt_full(x), q.tt_full(y), q.mpo_full(mpo)
    np.testing.assert_allclose(q.mpo_apply_dense(mpo, X), M @ X, rtol=1e-12, atol=1e-11)
    assert abs(q.tt_dot(x, y) - X @ Y) < 1e-12 * np.linalg.norm(X) * np.linalg.norm(Y)
    assert abs(q.tt_mpo_dot(y, mpo, x) - Y @ (M @ X)) < 1e-11 * np.linalg.norm(M @ X) * np.linalg.norm(Y)
    ref = (M @ Y) @ (M @ X)
    assert abs(q.tt_mpo_mpo_dot(y, mpo, mpo, x) - ref) < 1e-10 * abs(ref) + 1e-10
    D = q.mpo_full(q.diag_mpo(x))
    np.testing.assert_allclose(D, np.diag(X), atol=1e-13)


def test_left_canonical():
    x = random_mps_cores(9, 6, seed=7)
    lc = q.left_canonical(x)
    for c in lc[:-1]:
        m = c.reshape(-1, c.shape[2])
        np.testing.assert_allclose(m.T @ m, np.eye(m.shape[1]), atol=1e-13)
    np.testing.assert_allclose(q.tt_full(lc), q.tt_full(x), rtol=1e-12, atol=1e-13)
