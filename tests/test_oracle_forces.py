"""Pins of the body force G = rho g and the solid-phase velocity u_s of the
drag (Sec. 3.1) in the FP64 oracles (no GPU):

* hydrostatics: a closed column of liquid under gravity comes to rest with
  the pressure gradient rho g (2D and 3D);
* body-force Poiseuille flow between half-way bounce-back walls: the
  parabolic profile g (y + 1/2)(H - 1/2 - y) / (2 nu);
* a diffuse solid slab moving at u_s drags the liquid above it into Couette
  flow against a fixed wall: the slab's interior moves at u_s and the liquid
  profile is linear, vanishing at the wall.
"""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W, workloads3 as W3


def liquid_box(nx, ny, mat, phi0=None, periodic_x=True):
    z = np.zeros((ny, nx))
    return W.Case("box", nx, ny, periodic_x, False, [0, 0, 0, 0], {},
                  z.copy() if phi0 is None else phi0, z.copy(), np.ones((ny, nx)),
                  np.full((ny, nx), 0.5), mat)


def test_hydrostatic_column_2d(oracle_mod):
    """The column's sound waves decay as nu k^2: after 30000 steps of a
    32-node column the gradient is rho g to 1e-3 (64 nodes need 80000)."""
    mat = W.Material(g_y=-1e-5)
    o = oracle_mod.Oracle(liquid_box(4, 32, mat))
    o.step(30000)
    F = o.fields()
    p = F["p"][:, 1]
    y = np.arange(32, dtype=float)
    slope = np.polyfit(y[4:-4], p[4:-4], 1)[0]
    assert abs(slope / (mat.rho_l * mat.g_y) - 1.0) < 1e-3, slope
    assert np.abs(F["uy"]).max() < 1e-8


def test_hydrostatic_column_3d():
    from oracle import oracle3 as O3
    O3.build()
    mat = W.Material(g_z=-1e-5)
    n = (2, 2, 32)
    z = np.zeros((n[2], n[1], n[0]))
    case = W3.Case3("col3", *n, (True, True, False), [0] * 6, [0.0] * 6, z.copy(), z.copy(),
                    np.ones_like(z), np.full_like(z, 0.5), mat)
    o = O3.Oracle3(case)
    o.step(30000)
    F = o.fields()
    p = F["p"][:, 1, 1]
    zz = np.arange(n[2], dtype=float)
    slope = np.polyfit(zz[4:-4], p[4:-4], 1)[0]
    assert abs(slope / (mat.rho_l * mat.g_z) - 1.0) < 1e-3, slope
    assert np.abs(F["uz"]).max() < 1e-8


def test_body_force_poiseuille(oracle_mod):
    H = 32
    mat = W.Material(g_x=1e-6)
    o = oracle_mod.Oracle(liquid_box(4, H, mat))
    o.step(8000)
    u = o.fields()["ux"][:, 1]
    y = np.arange(H, dtype=float)
    nu = mat.mu_l / mat.rho_l
    exact = mat.g_x * (y + 0.5) * (H - 0.5 - y) / (2 * nu)
    assert np.abs(u - exact).max() < 0.01 * exact.max(), np.abs(u - exact).max() / exact.max()


def test_moving_slab_couette(oracle_mod):
    H, h_s, U = 48, 8.0, 1e-3
    mat = W.Material(us_x=U)
    y = np.arange(H, dtype=float)[:, None] * np.ones((1, 4))
    phi0 = W.slab_phi0(4, H, h_s, mat.eps)
    o = oracle_mod.Oracle(liquid_box(4, H, mat, phi0=phi0))
    o.step(20000)
    u = o.fields()["ux"][:, 1]
    # inside the slab, away from the fixed bounce-back wall below it
    assert np.abs(u[3:6] - U).max() < 1e-3 * U, u[3:6] / U
    core = slice(int(h_s) + 6, H - 4)
    yc = y[core, 0]
    fit = np.polyfit(yc, u[core], 1)
    resid = np.abs(np.polyval(fit, yc) - u[core]).max()
    assert resid < 5e-3 * U, resid / U
    assert fit[0] < 0 and abs(np.polyval(fit, H - 0.5)) < 0.05 * U    # zero at the fixed wall
