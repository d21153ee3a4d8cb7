"""Pins of the oracle's MRT flow collision (no GPU).

* the moment basis: rows are the energy, energy-square, momentum, energy-flux
  and stress polynomials evaluated at the printed D2Q9 velocities, mutually
  orthogonal with the known norms, and the inverse is an inverse;
* with every rate at the BGK rate the MRT step is the BGK step (freezing
  drop with flow, 150 steps), which checks the moment-space forcing and the
  generalised rest-population term of the pressure against the BGK forms;
* each non-conserved moment relaxes at its own rate: a lattice at rest
  perturbed along the energy-flux or a stress moment decays by exactly
  (1 - s) per step and stays in that moment;
* the shear viscosity is set by 1/tau_f alone: a shear wave decays at
  nu k^2 with nu = mu / rho whatever the other rates are;
* the static drop under MRT reaches the BGK drop's pressure jump (the
  equilibrium cannot depend on the rates) within the 2D Laplace law's bar:
  this checks the pressure recovery with a bulk rate away from 1/tau_f;
* phase field: a perturbation of g along any moment but the zeroth decays
  by exactly (1 - s) per step, s = 1/tau_g for the first moments and s_g
  above (the first moment of g does not feed the velocity); the flat
  interface stays the model's equilibrium under MRT.
"""

import ctypes as C
import math

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def polynomials():
    c2 = CX * CX + CY * CY
    return np.array([np.ones(9), -4 + 3 * c2, 4 - 10.5 * c2 + 4.5 * c2 * c2, CX, (-5 + 3 * c2) * CX,
                     CY, (-5 + 3 * c2) * CY, CX * CX - CY * CY, CX * CY])


def test_basis_and_inverse(oracle_mod):
    L = oracle_mod.lib()
    M = np.zeros(81)
    L.orc_mrt_matrix(_dp(M))
    M = M.reshape(9, 9)
    assert np.array_equal(M, polynomials())
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0
    assert np.array_equal(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])
    Mi = np.zeros(81)
    L.orc_invert9(_dp(np.ascontiguousarray(M.ravel())), _dp(Mi))
    assert np.abs(Mi.reshape(9, 9) @ M - np.eye(9)).max() < 1e-14


def _drop(mat):
    case = W.small_freezing_case()
    case.mat = mat
    return case


def test_equal_rates_reduce_to_bgk(oracle_mod):
    a = oracle_mod.Oracle(_drop(W.Material()))
    b = oracle_mod.Oracle(_drop(W.Material(mrt=1)))
    a.step(150)
    b.step(150)
    Fa, Fb = a.fields(), b.fields()
    assert np.abs(Fa["ux"]).max() > 1e-5 and Fa["fs"].max() > 0.1
    for k in ("phi", "T", "ux", "uy", "p", "fs"):
        assert np.abs(Fa[k] - Fb[k]).max() < 1e-12 * max(1.0, np.abs(Fa[k]).max()), k


def _rest_lattice(oracle_mod, mat, n=4):
    z = np.zeros((n, n))
    case = W.Case("rest", n, n, True, True, [0, 0, 0, 0], {}, z.copy(), z.copy(), np.ones((n, n)),
                  np.full((n, n), 0.5), mat)
    return oracle_mod.Oracle(case)


@pytest.mark.parametrize("row, rate", [(4, "q"), (6, "q"), (7, "nu"), (8, "nu")])
def test_moment_relaxes_at_its_rate(oracle_mod, row, rate):
    mat = W.Material(mrt=1, s_b=1.5, s_q=1.15)
    o = _rest_lattice(oracle_mod, mat)
    f, g, h, lag = o.get_state()
    delta = 1e-6
    f = f + delta * polynomials()[row][:, None, None]
    o.set_state(f, g, h, lag)
    o.step(1)
    f1 = o.get_state()[0]
    s = mat.s_q if rate == "q" else 1.0 / (3.0 * mat.mu_l / mat.rho_l + 0.5)
    expect = (1.0 - s) * delta * polynomials()[row][:, None, None]
    assert np.abs(f1 - expect).max() < 1e-18, (row, np.abs(f1 - expect).max())


@pytest.mark.parametrize("mat", [W.Material(), W.Material(mrt=1, s_b=1.6, s_q=1.1)],
                         ids=["bgk", "mrt"])
def test_shear_wave_viscosity(oracle_mod, mat):
    nx, ny, U = 4, 64, 1e-4
    k = 2 * math.pi / ny
    y = np.arange(ny, dtype=float)
    ux = U * np.sin(k * y)[:, None] * np.ones((1, nx))
    o = _rest_lattice(oracle_mod, mat)
    z = np.zeros((ny, nx))
    case = W.Case("shear", nx, ny, True, True, [0, 0, 0, 0], {}, z.copy(), z.copy(),
                  np.ones((ny, nx)), np.full((ny, nx), 0.5), mat)
    o = oracle_mod.Oracle(case)
    f, g, h, lag = o.get_state()
    L = oracle_mod.lib()
    out = np.zeros(9)
    for j in range(ny):
        L.orc_feq(0.0, mat.rho_l, float(ux[j, 0]), 0.0, _dp(out))
        f[:, j, :] = out[:, None]
    lag[2] = ux            # phi u of the previous step (phi = 1)
    lag[5] = ux            # and the velocity of the previous step
    o.set_state(f, g, h, lag)

    def amp():
        u = o.fields()["ux"][:, 0]
        return float(np.sum(u * np.sin(k * y)) / np.sum(np.sin(k * y) ** 2))

    o.step(100)
    a0 = amp()
    o.step(500)
    a1 = amp()
    nu = math.log(a0 / a1) / (500 * k * k)
    assert abs(nu / (mat.mu_l / mat.rho_l) - 1.0) < 0.01, nu


@pytest.mark.parametrize("row", range(1, 9))
def test_phase_field_moment_relaxes_at_its_rate(oracle_mod, row):
    mat = W.Material(mrt=1, s_b=1.5, s_q=1.15, s_g=1.35)
    o = _rest_lattice(oracle_mod, mat)
    f, g, h, lag = o.get_state()
    g0 = g.copy()
    delta = 1e-3            # g is O(1): the perturbation must stand well above its rounding
    o.set_state(f, g + delta * polynomials()[row][:, None, None], h, lag)
    o.step(1)
    g1 = o.get_state()[1]
    s = 1.0 / (3.0 * mat.mobility + 0.5) if row in (3, 5) else mat.s_g
    expect = g0 + (1.0 - s) * delta * polynomials()[row][:, None, None]
    assert np.abs(g1 - expect).max() < 1e-14, (row, np.abs(g1 - expect).max())


def test_flat_interface_stationary_under_mrt(oracle_mod):
    mat = W.Material(mrt=1, s_b=1.5, s_q=1.2, s_g=1.4)
    nx, ny = 4, 64
    yy = np.arange(ny, dtype=float)[:, None] * np.ones((1, nx))
    phi = np.tanh(2 * (yy - 15.5) / mat.eps) * np.tanh(2 * (47.5 - yy) / mat.eps)
    z = np.zeros((ny, nx))
    case = W.Case("flat_mrt", nx, ny, True, True, [0, 0, 0, 0], {}, z.copy(), z.copy(), phi,
                  np.ones((ny, nx)), mat)
    o = oracle_mod.Oracle(case)
    o.step(10000)
    assert np.abs(o.fields()["phi"] - phi).max() < 2e-2
    assert o.reduce()["umax"] < 1e-6


def test_laplace_law_under_mrt(oracle_mod):
    """8000 steps: BGK gives 0.9636 sigma/R here and the MRT drop (s_b 1.5,
    s_q 1.2) 0.9627, both converging to 0.9736 by 16000 steps; the phase
    field under MRT too (s_g 1.4)."""
    n, R = 80, 16.0
    mat = W.Material(mrt=1, s_b=1.5, s_q=1.2, s_g=1.4)
    yy, xx = np.mgrid[0:n, 0:n].astype(float)
    phi = np.tanh(2 * (R - np.hypot(xx - n / 2, yy - n / 2)) / mat.eps)
    z = np.zeros((n, n))
    case = W.Case("laplace_mrt", n, n, True, True, [0, 0, 0, 0], {}, z.copy(), z.copy(), phi,
                  np.ones((n, n)), mat)
    o = oracle_mod.Oracle(case)
    o.step(8000)
    F = o.fields()
    dp = F["p"][n // 2 - 3:n // 2 + 3, n // 2 - 3:n // 2 + 3].mean() - F["p"][:5, :5].mean()
    assert abs(dp / (mat.sigma / R) - 1.0) < 0.05, dp / (mat.sigma / R)
    assert o.reduce()["umax"] < 1e-5
