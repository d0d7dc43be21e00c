"""Dense-vector tensor-train reference (plain definitions of the TT operations).

Conventions (Sec. 2 and App. C/D of the paper):
* a TT-vector (MPS) of L cores A[k] with shapes (b_{k-1}, d, b_k), b_0 = b_L = 1,
  represents the vector whose entry at index sum_k r_k d^(L-k) is the product
  A[1]^{r_1} ... A[L]^{r_L}: the first core carries the most significant digit
  (App. D worked example);
* a TT-matrix (MPO) core has shape (w_{k-1}, 2 (out r'), 2 (in r), w_k) (Eq. simpleMatrix);
* a 2D field f_ij is encoded by a bit string of i and j (Sec. 3.2.1). "concatenated"
  is the paper's i_b then j_b; "interleaved" alternates i_1 j_1 i_2 j_2 ... (the
  ordering the library uses; both MSB first).

Every function here is the plain definition: dense arrays, numpy SVD/einsum, no
blocking or fusion.
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------
# bit-order maps (Sec. 3.2.1, App. C)
# ----------------------------------------------------------------------------

def qtt_index(i, j, n_eta, n_xi, order="interleaved"):
    """Position of grid point (i, j) in the dense QTT-ordered vector (MSB first)."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    if order == "concatenated":
        return (i << n_xi) | j
    if order != "interleaved":
        raise ValueError(order)
    if n_eta != n_xi:
        raise ValueError("interleaved order needs n_eta == n_xi")
    idx = np.zeros(np.broadcast(i, j).shape, dtype=np.int64)
    for m in range(n_eta):                      # m = 0 is the most significant bit
        ib = (i >> (n_eta - 1 - m)) & 1
        jb = (j >> (n_xi - 1 - m)) & 1
        idx = (idx << 2) | (ib << 1) | jb
    return idx


def grid_to_qtt(field, order="interleaved"):
    """(N_eta, N_xi) grid array -> dense vector in QTT order."""
    Ne, Nx = field.shape
    n_eta, n_xi = int(np.log2(Ne)), int(np.log2(Nx))
    ii, jj = np.meshgrid(np.arange(Ne), np.arange(Nx), indexing="ij")
    out = np.empty(Ne * Nx, dtype=field.dtype)
    out[qtt_index(ii, jj, n_eta, n_xi, order).ravel()] = field.ravel()
    return out


def qtt_to_grid(vec, n_eta, n_xi, order="interleaved"):
    ii, jj = np.meshgrid(np.arange(2 ** n_eta), np.arange(2 ** n_xi), indexing="ij")
    return vec[qtt_index(ii, jj, n_eta, n_xi, order)]


def grid_perm(n_eta, n_xi, order="interleaved"):
    """perm such that qtt_vec = grid_vec[perm] (grid_vec in row-major (i, j) order)."""
    ii, jj = np.meshgrid(np.arange(2 ** n_eta), np.arange(2 ** n_xi), indexing="ij")
    q = qtt_index(ii, jj, n_eta, n_xi, order).ravel()
    perm = np.empty_like(q)
    perm[q] = np.arange(q.size)
    return perm


# ----------------------------------------------------------------------------
# decompression, bond profile, NVPS (Eq. simpleMPS, Sec. 4)
# ----------------------------------------------------------------------------

def tt_full(cores):
    """Contract an MPS to its dense vector (first core = most significant digit)."""
    out = np.ones((1, 1))
    for c in cores:
        r0, d, r1 = c.shape
        out = (out @ c.reshape(r0, d * r1)).reshape(-1, r1)
    return out.reshape(-1)


def mpo_full(cores):
    """Dense matrix of an MPO: rows are output digits r', columns input digits r."""
    out = np.ones((1, 1, 1))           # (rows, cols, bond)
    for c in cores:
        w0, do, di, w1 = c.shape
        out = np.einsum("abw,wocx->aobcx", out, c).reshape(out.shape[0] * do, out.shape[1] * di, w1)
    return out[:, :, 0]


def bonds_of(cores):
    return [1] + [c.shape[-1] for c in cores]


def nvps(bonds, d=2):
    """Number of values parameterising a TT-vector: d * sum_k b_{k-1} b_k (Sec. 4)."""
    return int(d * sum(bonds[k] * bonds[k + 1] for k in range(len(bonds) - 1)))


def bond_cap_profile(L, chi, d=2):
    """dim(alpha_k) = min(d^k, d^(L-k), chi) (Eq. simpleMPS)."""
    return [int(min(d ** k, d ** (L - k), chi)) for k in range(L + 1)]


# ----------------------------------------------------------------------------
# TT-SVD (Sec. 2, successive SVDs; truncation: the smallest rank whose discarded
# singular values have Frobenius norm <= delta, capped at chi_max)
# ----------------------------------------------------------------------------

def choose_rank(s, delta, chi_max):
    """Smallest r with sqrt(sum_{i >= r} s_i^2) <= delta, then capped at chi_max (>= 1)."""
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]      # tail[r] = ||s[r:]||
    r = len(s)
    for k in range(len(s)):
        if tail[k] <= delta:
            r = k
            break
    return max(1, min(r, chi_max))


def tt_svd(vec, L, d=2, tol=0.0, chi_max=None, rule="rel"):
    """Decompose a dense vector of length d^L into an MPS by successive SVDs.

    rule "rel": per-bond discarded norm delta = tol/sqrt(L-1) * ||vec||, which gives
    ||vec - TT|| <= tol ||vec|| (quasi-optimality of TT-SVD).
    rule "abs": drop singular values below tol * (largest singular value at that bond).
    The bond is then capped at chi_max.
    """
    vec = np.asarray(vec, dtype=np.float64)
    chi_max = chi_max if chi_max is not None else 1 << 62
    nrm = np.linalg.norm(vec)
    delta = tol / np.sqrt(max(L - 1, 1)) * nrm
    cores = []
    C = vec.reshape(1, -1)
    r = 1
    for k in range(L - 1):
        C = C.reshape(r * d, -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        if rule == "rel":
            rk = choose_rank(s, delta, chi_max)
        else:
            keep = int(np.sum(s > tol * (s[0] if s.size else 0.0)))
            rk = max(1, min(keep, chi_max))
        cores.append(U[:, :rk].reshape(r, d, rk))
        C = s[:rk, None] * Vt[:rk]
        r = rk
    cores.append(C.reshape(r, d, 1))
    return cores


def tt_round_dense(cores, tol=0.0, chi_max=None):
    """Reference rounding: TT-SVD of the decompressed vector (same rule as tt_svd)."""
    L = len(cores)
    d = cores[0].shape[1]
    return tt_svd(tt_full(cores), L, d, tol, chi_max)


# ----------------------------------------------------------------------------
# operator action, inner products (Sec. 2.1)
# ----------------------------------------------------------------------------

def mpo_apply_dense(mpo, vec):
    """y = M x for a dense vector x, applying the MPO site by site (Sec. 2.1.2).

    Memory is w * 2^L; the result equals mpo_full(mpo) @ vec.
    """
    L = len(mpo)
    T = np.asarray(vec, dtype=np.float64).reshape(1, 1, -1)       # (done-out, bond, remaining-in)
    for k in range(L):
        P, b, R = T.shape
        T = T.reshape(P, b, 2, R // 2)
        T = np.einsum("pbsr,bosc->pocr", T, mpo[k]).reshape(P * 2, mpo[k].shape[3], R // 2)
    return T.reshape(-1)


def tt_dot(x, y):
    """<x, y> of two MPS by left environments E_k = sum_r X^r^T E_{k-1} Y^r."""
    E = np.ones((1, 1))
    for a, b in zip(x, y):
        E = np.einsum("ij,isk,jsl->kl", E, a, b)
    return float(E[0, 0])


def tt_mpo_dot(x, mpo, y):
    """<x, M y> by environments of shape (bx, w, by)."""
    E = np.ones((1, 1, 1))
    for a, m, b in zip(x, mpo, y):
        E = np.einsum("iwj,iok,wosv,jsl->kvl", E, a, m, b)
    return float(E[0, 0, 0])


def tt_mpo_mpo_dot(x, m1, m2, y):
    """<M1 x, M2 y> = <x, M1^T M2 y> by environments of shape (bx, w1, w2, by)."""
    E = np.ones((1, 1, 1, 1))
    for a, p, q, b in zip(x, m1, m2, y):
        E = np.einsum("iuvj,isk,uosa,votb,jtl->kabl", E, a, p, q, b)
    return float(E[0, 0, 0, 0])


def left_canonical(cores):
    """QR sweep left to right: every core but the last becomes left-orthonormal."""
    out = [c.copy() for c in cores]
    for k in range(len(out) - 1):
        r0, d, r1 = out[k].shape
        Q, R = np.linalg.qr(out[k].reshape(r0 * d, r1))
        out[k] = Q.reshape(r0, d, Q.shape[1])
        out[k + 1] = np.einsum("ij,jsk->isk", R, out[k + 1])
    return out


def diag_mpo(cores):
    """Diagonal TT-matrix of an MPS via the copy tensor (Sec. 2.1.3)."""
    out = []
    for c in cores:
        r0, d, r1 = c.shape
        m = np.zeros((r0, d, d, r1))
        for s in range(d):
            m[:, s, s, :] = c[:, s, :]
        out.append(m)
    return out


def app_d_cores():
    """The worked example of App. D: three cores whose product is t = (1, ..., 8)."""
    A1 = np.zeros((1, 2, 2)); A1[0, :, 0] = [1, 1]; A1[0, :, 1] = [0, 1]
    A2 = np.zeros((2, 2, 2))
    A2[0, :, 0] = [1, 1]; A2[0, :, 1] = [0, 1]
    A2[1, :, 0] = [0, 0]; A2[1, :, 1] = [2, 2]
    A3 = np.zeros((2, 2, 1)); A3[0, :, 0] = [1, 2]; A3[1, :, 0] = [2, 2]
    return [A1, A2, A3]
