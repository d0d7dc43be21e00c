"""O-grid around a unit-diameter cylinder and its discrete metric terms.

Follows App. E (Eq. mesh) for the points and App. A for the metrics:
  x_ij = (D/2) (D_outer/D)^((i+1)/(N_eta+1)) cos(2 pi j dxi),  z likewise with sin,
  i = -1 .. N_eta (i = -1 is the cylinder wall, i = N_eta the outer boundary),
  j periodic, d_eta = 1/(N_eta+1), d_xi = 1/N_xi.
Metric derivatives are second-order central differences in the computational
coordinates (App. A), periodic in xi.

Reading where the paper leaves a choice open: metric terms at the two boundary rows need one
more row of points on each side; those rows are taken from the same mesh formula
evaluated at i = -2 and i = N_eta + 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class OGrid:
    n_eta: int
    n_xi: int
    r_out: float = 20.0     # outer radius (D = 1, so D_outer / D = 2 r_out)
    r_in: float = 0.5       # cylinder radius D/2

    def __post_init__(self):
        self.N_eta = 2 ** self.n_eta
        self.N_xi = 2 ** self.n_xi
        self.d_eta = 1.0 / (self.N_eta + 1)
        self.d_xi = 1.0 / self.N_xi
        # rows i = -2 .. N_eta+1 (extended by one row each side for metric terms)
        self.i_ext = np.arange(-2, self.N_eta + 2)
        ratio = (2.0 * self.r_out) / (2.0 * self.r_in)
        self.r_ext = self.r_in * ratio ** ((self.i_ext + 1) * self.d_eta)
        j = np.arange(self.N_xi)
        self.theta = 2.0 * np.pi * j * self.d_xi
        self.x_ext = self.r_ext[:, None] * np.cos(self.theta)[None, :]
        self.z_ext = self.r_ext[:, None] * np.sin(self.theta)[None, :]
        self._metrics()

    # rows of the "boundary-inclusive" array: i = -1 .. N_eta  -> ext rows 1 .. N_eta+2
    @property
    def r_bnd(self):
        """Radii of rows i = -1 .. N_eta."""
        return self.r_ext[1:-1]

    @property
    def r_int(self):
        """Radii of interior rows i = 0 .. N_eta-1."""
        return self.r_ext[2:-2]

    def _dxi(self, f):
        """Central difference in xi (periodic), App. A."""
        return (np.roll(f, -1, axis=1) - np.roll(f, 1, axis=1)) / (2.0 * self.d_xi)

    def _deta(self, f):
        """Central difference in eta on rows 1..n-2 of f (drops one row on each side), App. A."""
        return (f[2:, :] - f[:-2, :]) / (2.0 * self.d_eta)

    def _metrics(self):
        # metric terms on rows i = -1 .. N_eta  (N_eta + 2 rows)
        x, z = self.x_ext, self.z_ext
        self.x_xi = self._dxi(x)[1:-1]
        self.z_xi = self._dxi(z)[1:-1]
        self.x_eta = self._deta(x)
        self.z_eta = self._deta(z)
        # Jacobian determinant and metric tensor (App. A)
        self.J = self.x_xi * self.z_eta - self.x_eta * self.z_xi
        self.g11 = self.x_xi ** 2 + self.z_xi ** 2
        self.g22 = self.x_eta ** 2 + self.z_eta ** 2
        self.g12 = self.x_xi * self.x_eta + self.z_xi * self.z_eta

    def interior(self, a):
        """Restrict a boundary-inclusive (N_eta+2, N_xi) array to interior rows."""
        return a[1:-1]

    def h_min(self):
        """Smallest physical spacing at the wall: min(radial step, arc step) (Sec. 4)."""
        radial = self.r_ext[2] - self.r_ext[1]          # row 0 minus wall row -1
        arc = 2.0 * np.pi * self.r_in * self.d_xi
        return min(radial, arc)

    def closed_form(self):
        """Closed-form metrics of this exponential O-grid (derived from App. A + Eq. mesh).

        c_xi = sin(2 pi d_xi)/d_xi, c_eta = sinh(lambda d_eta)/d_eta, lambda = ln(r_out/r_in):
        J = -r^2 c_xi c_eta, g11 = r^2 c_xi^2, g22 = r^2 c_eta^2, g12 = 0.
        """
        lam = np.log(self.r_out / self.r_in)
        c_xi = np.sin(2.0 * np.pi * self.d_xi) / self.d_xi
        c_eta = np.sinh(lam * self.d_eta) / self.d_eta
        r = self.r_bnd[:, None] * np.ones((1, self.N_xi))
        return dict(c_xi=c_xi, c_eta=c_eta, J=-r ** 2 * c_xi * c_eta,
                    g11=r ** 2 * c_xi ** 2, g22=r ** 2 * c_eta ** 2, g12=np.zeros_like(r))
