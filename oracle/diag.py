"""Diagnostics of Sec. 4 and App. F: weighted L2 errors, forces, Strouhal number.

Readings where the paper leaves a choice open:
* the L2 weight is |J| (J < 0 on this grid orientation), Eq. (error);
* force on the body F = sum_j tau(x_j) n_j R 2 pi d_xi with n = (cos t, sin t)
  pointing into the fluid, R = D/2 (App. F); C = 2F (Eq. liftdrag, rho = U = D = 1);
* tau = -(p + 2/(3Re) div v) I + (1/Re)(grad v + grad v^T) (App. F, with its
  2/(3Re) term kept literally);
* wall values: p_wall = p_{0,j}; eta-derivatives one-sided second order from rows
  -1, 0, 1; xi-derivatives central along the wall from the prescribed wall velocity;
* Strouhal: upward crossings of C_L - mean(C_L) with linear interpolation over the
  window; St = 1/mean period (D = U = 1) (Sec. 4.1.2).
"""
from __future__ import annotations

import numpy as np

from .grid import OGrid


def l2_norm(g: OGrid, s):
    """||s||_L2 ~ sqrt(d_xi d_eta sum |s_ij|^2 |J_ij|) over the interior (Eq. error)."""
    J = np.abs(g.interior(g.J)).ravel()
    return float(np.sqrt(g.d_xi * g.d_eta * np.sum(np.abs(np.ravel(s)) ** 2 * J)))


def eps_l2(g: OGrid, s_tt, s_ref):
    return l2_norm(g, np.ravel(s_tt) - np.ravel(s_ref)) / l2_norm(g, s_ref)


def eps_max(s_tt, s_ref):
    return float(np.max(np.abs(np.ravel(s_tt) - np.ravel(s_ref))))


def kinetic_energy(g: OGrid, u, v):
    """E_kin = 1/2 ||v||_L2^2 (Sec. 4.1.1)."""
    return 0.5 * (l2_norm(g, u) ** 2 + l2_norm(g, v) ** 2)


def wall_derivs(g: OGrid, f_wall, f0, f1):
    """(d/dx f, d/dz f) at the wall row i = -1 from its values on rows -1, 0, 1."""
    f_xi = (np.roll(f_wall, -1) - np.roll(f_wall, 1)) / (2 * g.d_xi)
    f_eta = (-3.0 * f_wall + 4.0 * f0 - f1) / (2 * g.d_eta)
    # metric terms on row -1 (index 0 of the boundary-inclusive metric arrays)
    J = g.J[0]
    fx = (g.z_eta[0] * f_xi - g.z_xi[0] * f_eta) / J
    fz = (-g.x_eta[0] * f_xi + g.x_xi[0] * f_eta) / J
    return fx, fz


def forces(g: OGrid, u, v, p, Re, u_wall, v_wall):
    """(C_D, C_L) from interior fields (flattened grid order) and wall velocity (App. F)."""
    Ne, Nx = g.N_eta, g.N_xi
    U = np.reshape(u, (Ne, Nx)); V = np.reshape(v, (Ne, Nx)); P = np.reshape(p, (Ne, Nx))
    ux, uz = wall_derivs(g, u_wall, U[0], U[1])
    vx, vz = wall_derivs(g, v_wall, V[0], V[1])
    pw = P[0]
    div = ux + vz
    t11 = -(pw + 2.0 / (3.0 * Re) * div) + 2.0 / Re * ux
    t22 = -(pw + 2.0 / (3.0 * Re) * div) + 2.0 / Re * vz
    t12 = (uz + vx) / Re
    c, s = np.cos(g.theta), np.sin(g.theta)
    ds = g.r_in * 2.0 * np.pi * g.d_xi
    Fx = np.sum(t11 * c + t12 * s) * ds
    Fz = np.sum(t12 * c + t22 * s) * ds
    return 2.0 * Fx, 2.0 * Fz


def strouhal(t, cl, window=0.5, min_periods=3):
    """(St, lift amplitude) from a C_L(t) history; St is None if fewer than min_periods."""
    t = np.asarray(t, dtype=float); cl = np.asarray(cl, dtype=float)
    n0 = int(len(t) * (1.0 - window))
    t, cl = t[n0:], cl[n0:]
    y = cl - cl.mean()
    up = np.nonzero((y[:-1] < 0) & (y[1:] >= 0))[0]
    tc = t[up] - y[up] * (t[up + 1] - t[up]) / (y[up + 1] - y[up])
    amp = 0.5 * (cl.max() - cl.min())
    if len(tc) < min_periods + 1:
        return None, amp
    T = np.mean(np.diff(tc))
    return 1.0 / T, amp
