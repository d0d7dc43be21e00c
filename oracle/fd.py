"""Classical finite-difference twin of the scheme (the oracle's plain definition).

The paper implements the same fractional-step scheme twice, once in TT format and
once classically (Sec. 3.3 end, App. H); as the bond dimension grows the TT result
tends to this one. This module is that classical implementation, in FP64:

* computational-space stencils, second-order central (App. A);
* curvilinear first derivatives (App. A, Eq. curviliner-deriavtive) and the
  seven-term Laplacian taken literally (App. A);
* ghost-point boundaries (Sec. 3.1): every operator is an interior matrix plus a
  boundary-correction vector built from the boundary-row values;
  velocity: Dirichlet at the wall (row i=-1) and at the outer boundary (row N_eta);
  pressure: zero normal derivative at the wall, p = 0 at the outer boundary (Eq. bound);
* the Chorin fractional step, Eqs. (intermediate_vel_eq) and (Poisson) and the
  projection that follows them (Sec. 3.3), with the J-weighted Poisson system (Sec. 3.3).

Readings where the paper leaves a choice open: wall pressure ghost value p_{-1,j} = p_{0,j};
the J-weight uses |J| (J < 0 for this orientation); the viscous term is implicit
and convection explicit, as in Eq. (intermediate_vel_eq).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .grid import OGrid


# ----------------------------------------------------------------------------
# stencils on the boundary-inclusive grid (rows i = -1 .. N_eta), App. A
# ----------------------------------------------------------------------------

class Stencils:
    """Sparse maps from a boundary-inclusive field (N_eta+2)*N_xi -> interior N_eta*N_xi."""

    def __init__(self, g: OGrid):
        self.g = g
        Ne, Nx = g.N_eta, g.N_xi
        self.n_int = Ne * Nx
        self.n_ext = (Ne + 2) * Nx
        ii, jj = np.meshgrid(np.arange(Ne), np.arange(Nx), indexing="ij")
        self.ii, self.jj = ii.ravel(), jj.ravel()
        self.rows = np.arange(self.n_int)

    def ext(self, i, j):
        """Index of (i, j) in the boundary-inclusive vector; i in [-1, N_eta], j periodic."""
        return (i + 1) * self.g.N_xi + np.mod(j, self.g.N_xi)

    def _mat(self, terms):
        rows, cols, vals = [], [], []
        for di, dj, w in terms:
            rows.append(self.rows)
            cols.append(self.ext(self.ii + di, self.jj + dj))
            vals.append(np.full(self.n_int, w))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.n_int, self.n_ext))

    def d_xi(self):
        h = self.g.d_xi
        return self._mat([(0, 1, 1 / (2 * h)), (0, -1, -1 / (2 * h))])

    def d_eta(self):
        h = self.g.d_eta
        return self._mat([(1, 0, 1 / (2 * h)), (-1, 0, -1 / (2 * h))])

    def d_xixi(self):
        h = self.g.d_xi
        return self._mat([(0, 1, 1 / h ** 2), (0, 0, -2 / h ** 2), (0, -1, 1 / h ** 2)])

    def d_etaeta(self):
        h = self.g.d_eta
        return self._mat([(1, 0, 1 / h ** 2), (0, 0, -2 / h ** 2), (-1, 0, 1 / h ** 2)])

    def d_xieta(self):
        c = 1.0 / (4 * self.g.d_xi * self.g.d_eta)
        return self._mat([(1, 1, c), (1, -1, -c), (-1, 1, -c), (-1, -1, c)])


def _diag(a):
    return sp.diags(np.ravel(a))


class CurvilinearOps:
    """Curvilinear operators of App. A as maps boundary-inclusive -> interior."""

    def __init__(self, g: OGrid):
        self.g = g
        s = self.s = Stencils(g)
        Dxi, Deta = s.d_xi(), s.d_eta()
        I = g.interior
        J = I(g.J)
        # first derivatives, Eq. (curviliner-deriavtive)
        self.Dx_ext = (_diag(I(g.z_eta) / J) @ Dxi - _diag(I(g.z_xi) / J) @ Deta).tocsr()
        self.Dz_ext = (-_diag(I(g.x_eta) / J) @ Dxi + _diag(I(g.x_xi) / J) @ Deta).tocsr()
        # seven-term Laplacian, App. A (coefficients on rows -1..N_eta, derivatives by
        # central differences at the interior rows)
        a22 = g.g22 / g.J          # rows -1..N_eta
        a11 = g.g11 / g.J
        a12 = g.g12 / g.J
        dxi = lambda f: I(g._dxi(f))
        deta = lambda f: g._deta(f)
        terms = (_diag(dxi(a22)) @ Dxi
                 + _diag(I(a22)) @ s.d_xixi()
                 - _diag(dxi(a12)) @ Deta
                 - _diag(deta(a12)) @ Dxi
                 - 2.0 * _diag(I(a12)) @ s.d_xieta()
                 + _diag(deta(a11)) @ Deta
                 + _diag(I(a11)) @ s.d_etaeta())
        self.Lap_ext = (_diag(1.0 / J) @ terms).tocsr()
        self.absJ = np.abs(J).ravel()

    # -- splitting into interior / boundary columns (ghost-point approach, Sec. 3.1)
    def _split(self, A):
        Nx, Ne = self.g.N_xi, self.g.N_eta
        A = A.tocsc()
        A_wall = A[:, 0:Nx]
        A_int = A[:, Nx:(Ne + 1) * Nx]
        A_out = A[:, (Ne + 1) * Nx:]
        return A_int.tocsr(), A_wall.tocsr(), A_out.tocsr()

    def velocity_op(self, A_ext):
        """(A_int, bc(wall_vals, outer_vals)) for a Dirichlet-Dirichlet field."""
        A_int, A_wall, A_out = self._split(A_ext)
        def bc(wall, outer):
            return A_wall @ np.broadcast_to(wall, (self.g.N_xi,)) + A_out @ np.broadcast_to(outer, (self.g.N_xi,))
        return A_int, bc

    def pressure_op(self, A_ext):
        """Interior matrix with p_{-1,j} = p_{0,j} folded in and p_{N_eta,j} = 0."""
        A_int, A_wall, _ = self._split(A_ext)
        Nx, n = self.g.N_xi, self.s.n_int
        # E maps the wall value of column j to interior unknown (0, j)
        E = sp.csr_matrix((np.ones(Nx), (np.arange(Nx), np.arange(Nx))), shape=(Nx, n))
        return (A_int + A_wall @ E).tocsr()


# ----------------------------------------------------------------------------
# boundary data (Eq. bound, Eq. rot_bc)
# ----------------------------------------------------------------------------

def velocity_bc(g: OGrid, alpha: float = 0.0, u_inf: float = 1.0):
    """Wall and far-field values for u and v. Wall: Eq. (rot_bc) with rate alpha
    (alpha = 0 is the no-slip non-rotating wall); far field: v = (u_inf, 0)."""
    th = g.theta
    return dict(u_wall=alpha * np.sin(th), v_wall=-alpha * np.cos(th),
                u_out=np.full(g.N_xi, u_inf), v_out=np.zeros(g.N_xi))


# ----------------------------------------------------------------------------
# the fractional step, Sec. 3.3
# ----------------------------------------------------------------------------

class FDSolver:
    """Dense-grid fractional step with sparse-LU solves (factorised once)."""

    def __init__(self, g: OGrid, Re: float, dt: float, alpha: float = 0.0, solver: str = "lu"):
        """solver: "lu" (sparse LU of the literal seven-term operators) or "fft" (the
        independent closed-form FFT/Thomas solvers, which agree with LU to round-off)."""
        self.g, self.Re, self.dt, self.alpha, self.solver = g, Re, dt, alpha, solver
        ops = self.ops = CurvilinearOps(g)
        self.Dx, self.bcx = ops.velocity_op(ops.Dx_ext)
        self.Dz, self.bcz = ops.velocity_op(ops.Dz_ext)
        self.Lap, self.bcL = ops.velocity_op(ops.Lap_ext)
        self.Dx_p = ops.pressure_op(ops.Dx_ext)
        self.Dz_p = ops.pressure_op(ops.Dz_ext)
        self.Lap_p = ops.pressure_op(ops.Lap_ext)
        self.bc = velocity_bc(g, alpha)
        n = ops.s.n_int
        c = dt / Re
        self.H = (sp.identity(n) - c * self.Lap).tocsc()
        self.P = (-_diag(ops.absJ) @ self.Lap_p).tocsc()      # J-weighted SPD form
        self._luH = None
        self._luP = None

    def luH(self):
        if self._luH is None:
            self._luH = spla.splu(self.H)
        return self._luH

    def luP(self):
        if self._luP is None:
            self._luP = spla.splu(self.P)
        return self._luP

    def grads(self, u, v):
        b = self.bc
        return dict(gxu=self.Dx @ u + self.bcx(b["u_wall"], b["u_out"]),
                    gzu=self.Dz @ u + self.bcz(b["u_wall"], b["u_out"]),
                    gxv=self.Dx @ v + self.bcx(b["v_wall"], b["v_out"]),
                    gzv=self.Dz @ v + self.bcz(b["v_wall"], b["v_out"]))

    def step(self, u, v, return_stages=False):
        """One step from interior fields u, v (flattened grid order) -> u, v, p."""
        b, dt, Re = self.bc, self.dt, self.Re
        gr = self.grads(u, v)
        conv_u = u * gr["gxu"] + v * gr["gzu"]          # (v . grad) u
        conv_v = u * gr["gxv"] + v * gr["gzv"]
        rhs_u = u - dt * conv_u + (dt / Re) * self.bcL(b["u_wall"], b["u_out"])
        rhs_v = v - dt * conv_v + (dt / Re) * self.bcL(b["v_wall"], b["v_out"])
        if self.solver == "fft":
            us = fast_helmholtz(self.g, dt / Re, rhs_u)  # Eq. (intermediate_vel_eq)
            vs = fast_helmholtz(self.g, dt / Re, rhs_v)
        else:
            us = self.luH().solve(rhs_u)                 # Eq. (intermediate_vel_eq)
            vs = self.luH().solve(rhs_v)
        div = (self.Dx @ us + self.bcx(b["u_wall"], b["u_out"])
               + self.Dz @ vs + self.bcz(b["v_wall"], b["v_out"])) / dt
        if self.solver == "fft":
            p = fast_poisson(self.g, -self.ops.absJ * div)
        else:
            p = self.luP().solve(-self.ops.absJ * div)  # Eq. (Poisson), J-weighted
        un = us - dt * (self.Dx_p @ p)
        vn = vs - dt * (self.Dz_p @ p)
        if return_stages:
            st = dict(gr)
            st.update(conv_u=conv_u, conv_v=conv_v, rhs_u=rhs_u, rhs_v=rhs_v,
                      us=us, vs=vs, div=div, p=p, u=un, v=vn)
            return st
        return un, vn, p


# ----------------------------------------------------------------------------
# an independent fast solver for the separable closed form (FFT in xi, Thomas in eta)
# ----------------------------------------------------------------------------

def _thomas(a, b, c, d):
    """Solve tridiagonal systems (batched over the last axis): a sub, b diag, c super."""
    n = b.shape[0]
    cp = np.empty_like(d)
    dp = np.empty_like(d)
    bb = np.array(b, dtype=d.dtype)
    cp[0] = c[0] / bb[0]
    dp[0] = d[0] / bb[0]
    for i in range(1, n):
        m = bb[i] - a[i] * cp[i - 1]
        cp[i] = (c[i] / m) if i < n - 1 else 0.0
        dp[i] = (d[i] - a[i] * dp[i - 1]) / m
    x = np.empty_like(d)
    x[-1] = dp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def fast_poisson(g: OGrid, rhs):
    """Solve (-|J| Lap_p) p = rhs with the closed-form metrics of the O-grid.

    On this grid |J| Lap = (c_eta/c_xi) d2_xi + (c_xi/c_eta) d2_eta (constant
    coefficients), so a DFT in the periodic xi direction leaves one tridiagonal
    system in eta per mode; the wall row uses p_{-1} = p_0, the outer row p = 0.
    """
    cf = g.closed_form()
    a_xi = cf["c_eta"] / cf["c_xi"] / g.d_xi ** 2
    a_eta = cf["c_xi"] / cf["c_eta"] / g.d_eta ** 2
    Ne, Nx = g.N_eta, g.N_xi
    R = np.fft.fft(rhs.reshape(Ne, Nx), axis=1)
    k = np.arange(Nx)
    lam_xi = 4.0 * a_xi * np.sin(np.pi * k / Nx) ** 2        # eigenvalues of -a_xi d2_xi
    sub = np.full((Ne, 1), -a_eta)
    sup = np.full((Ne, 1), -a_eta)
    diag = np.full((Ne, Nx), 2.0 * a_eta) + lam_xi[None, :]
    diag[0, :] -= a_eta                                      # Neumann fold at the wall row
    P = _thomas(np.broadcast_to(sub, (Ne, Nx)), diag, np.broadcast_to(sup, (Ne, Nx)), R.astype(complex))
    return np.real(np.fft.ifft(P, axis=1)).ravel()


def fast_helmholtz(g: OGrid, c, rhs):
    """Solve (I - c Lap) u = rhs (Dirichlet rows -1 and N_eta folded into rhs already)
    with the closed form Lap = d2_xi/(r^2 c_xi^2) + d2_eta/(r^2 c_eta^2)."""
    cf = g.closed_form()
    Ne, Nx = g.N_eta, g.N_xi
    r2 = g.r_int ** 2
    R = np.fft.fft(rhs.reshape(Ne, Nx), axis=1)
    k = np.arange(Nx)
    lam_xi = 4.0 * np.sin(np.pi * k / Nx) ** 2 / g.d_xi ** 2 / cf["c_xi"] ** 2   # -d2_xi / c_xi^2
    ae = c / (r2 * cf["c_eta"] ** 2 * g.d_eta ** 2)                            # per row
    diag = 1.0 + c * lam_xi[None, :] / r2[:, None] + 2.0 * ae[:, None]
    sub = np.broadcast_to(-ae[:, None], (Ne, Nx))
    P = _thomas(sub, diag, sub, R.astype(complex))
    return np.real(np.fft.ifft(P, axis=1)).ravel()


# ----------------------------------------------------------------------------
# initial fields
# ----------------------------------------------------------------------------

def uniform_flow(g: OGrid, u_inf: float = 1.0):
    n = g.N_eta * g.N_xi
    return np.full(n, u_inf), np.zeros(n)


def perturbation(g: OGrid, A0: float):
    """Transient trigger of App. G (Eq. init_cond), read as vanishing towards the far
    field (the text's stated intent): A0 (e^{(1-(i+1) d_eta)^6} - 1)/(e - 1) sin(2 pi j d_xi)."""
    i = np.arange(g.N_eta)
    env = (np.exp((1.0 - (i + 1) * g.d_eta) ** 6) - 1.0) / (np.e - 1.0)
    return (A0 * env[:, None] * np.sin(g.theta)[None, :]).ravel()
