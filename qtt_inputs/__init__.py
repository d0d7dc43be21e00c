"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only draws random numbers and fixes array shapes; it contains none
of the method's arithmetic (no decompositions, no operators, no contractions).
Both the CPU oracle and the GPU library receive exactly these arrays, so the two
sides start from identical data.

Shapes follow the tensor-train conventions of the paper (Sec. 2): an MPS core is
(chi_{k-1}, 2, chi_k), an MPO core is (w_{k-1}, 2 (out), 2 (in), w_k), and the
bond profile of an untruncated train is min(2^k, 2^(L-k), chi) (Eq. simpleMPS).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "bond_profile",
    "noise_fields",
    "random_mps_cores",
    "random_mpo_cores",
    "rotating_samples",
]


def bond_profile(L: int, chi: int, d: int = 2) -> list[int]:
    """Capacity bond profile dim(alpha_k) = min(d^k, d^(L-k), chi), k = 0..L (Eq. simpleMPS)."""
    out = []
    for k in range(L + 1):
        out.append(int(min(d ** k, d ** (L - k), chi)))
    return out


def noise_fields(n_eta: int, n_xi: int, sigma: float, seed: int = 0) -> np.ndarray:
    """Gaussian noise for (u, v) on the N_eta x N_xi interior grid, grid (i, j) order.

    Returns an array of shape (2, 2**n_eta, 2**n_xi): index 0 is u, index 1 is v.
    """
    rng = np.random.default_rng(seed)
    return rng.standard_normal((2, 2 ** n_eta, 2 ** n_xi)) * sigma


def random_mps_cores(L: int, chi: int, seed: int, d: int = 2) -> list[np.ndarray]:
    """Cores with i.i.d. N(0, 1/chi) entries on the capacity bond profile.

    Core k has shape (b[k], d, b[k+1]) with b = bond_profile(L, chi, d).
    """
    rng = np.random.default_rng(seed)
    b = bond_profile(L, chi, d)
    scale = 1.0 / np.sqrt(chi)
    return [rng.standard_normal((b[k], d, b[k + 1])) * scale for k in range(L)]


def random_mpo_cores(L: int, w: int, seed: int) -> list[np.ndarray]:
    """MPO cores with i.i.d. N(0, 1) entries, bond w inside and 1 at both ends.

    Core k has shape (w_{k}, 2, 2, w_{k+1}) laid out as [left][out][in][right].
    """
    rng = np.random.default_rng(seed)
    wb = [1] + [w] * (L - 1) + [1]
    return [rng.standard_normal((wb[k], 2, 2, wb[k + 1])) for k in range(L)]


def rotating_samples(n: int, seed: int) -> np.ndarray:
    """(Re, alpha) pairs: Re ~ U[60, 200], rotation rate alpha ~ U[0, 2]; shape (n, 2)."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(60.0, 200.0, size=n)
    al = rng.uniform(0.0, 2.0, size=n)
    return np.stack([re, al], axis=1)
