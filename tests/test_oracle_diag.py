"""Pins of the oracle diagnostics (forces, Strouhal number, weighted norms)."""
import numpy as np

from oracle import diag
from oracle.grid import OGrid


def test_pressure_force_closed_form():
    """p = z, v = 0: F = -sum p n ds with p_wall = p_{0,j} = r_0 sin t -> C_L = -pi r_0 (trapezoid exact)."""
    g = OGrid(6, 6)
    n = g.N_eta * g.N_xi
    Z = g.z_ext[2:-2].ravel()
    cd, cl = diag.forces(g, np.zeros(n), np.zeros(n), Z, 100.0, np.zeros(g.N_xi), np.zeros(g.N_xi))
    assert abs(cl + np.pi * g.r_int[0]) < 1e-12
    assert abs(cd) < 1e-12


def test_rigid_rotation_has_no_viscous_force():
    """u = -w z, v = w x is a rigid motion: zero strain, so zero viscous stress and div."""
    g = OGrid(6, 6)
    w = 0.7
    U = (-w * g.z_ext[2:-2]).ravel(); V = (w * g.x_ext[2:-2]).ravel()
    uw = -w * g.z_ext[1]; vw = w * g.x_ext[1]
    cd, cl = diag.forces(g, U, V, np.zeros_like(U), 10.0, uw, vw)
    assert abs(cd) < 1e-4 and abs(cl) < 1e-4


def test_viscous_shear_force():
    """u = z^2, v = 0: tau_12 = 2z/Re at the wall, C_D = 4 pi R^2 / Re (second-order discretisation)."""
    g = OGrid(8, 8, r_out=4.0)
    Re = 10.0
    U = (g.z_ext[2:-2] ** 2).ravel()
    cd, cl = diag.forces(g, U, np.zeros_like(U), np.zeros_like(U), Re, g.z_ext[1] ** 2, np.zeros(g.N_xi))
    ref = 4 * np.pi * 0.25 / Re
    assert abs(cd - ref) < 2e-3 * ref, (cd, ref)
    assert abs(cl) < 1e-10


def test_strouhal_from_sinusoid():
    t = np.linspace(0.0, 100.0, 50001)
    st, amp = diag.strouhal(t, 2.49 + 0.3 * np.sin(2 * np.pi * 0.1663 * t + 0.4))
    assert abs(st - 0.1663) < 1e-6 and abs(amp - 0.3) < 1e-4
    st2, _ = diag.strouhal(t[:500], np.sin(2 * np.pi * 0.1 * t[:500]))
    assert st2 is None


def test_l2_weight_integrates_annulus_area():
    """sum |J| d_xi d_eta approximates the physical area pi (R_out^2 - R_in^2) to O(h^2)."""
    g = OGrid(9, 9)
    area = diag.l2_norm(g, np.ones(g.N_eta * g.N_xi)) ** 2
    ref = np.pi * (20.0 ** 2 - 0.5 ** 2)
    assert abs(area - ref) < 2e-2 * ref
    assert diag.eps_l2(g, 1.01 * np.ones(g.N_eta * g.N_xi), np.ones(g.N_eta * g.N_xi)) - 0.01 < 1e-12
