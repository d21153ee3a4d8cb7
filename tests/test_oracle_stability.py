"""Linear stability of the oracle's TRT enthalpy scheme (Sec. 3.3, eq22, with
readings R4 and R5): the basis of reading R6, which bounds the reference heat
capacity rho_ref C_p,ref by the smallest nodal heat capacity rho C_p.

Von Neumann analysis at rest (u = 0, no phase change, one material): a
perturbation of the populations changes rho H = sum h and T = rho H / (rho C_p);
the oracle's own equilibrium (orc_heq) gives the linear map h -> h^eq, the TRT
collision relaxes its antisymmetric part at 1/tau_a and its symmetric part at
1/tau_s (1/tau_s + 1/tau_a = 2), and streaming multiplies population i of a
Fourier mode exp(i k.x) by exp(-i k.c_i).  The growth factor of the step is
the largest eigenvalue modulus over all wave vectors.  It is exactly 1 (the
conserved mode) while rho C_p >= w_0 rho_ref C_p,ref = 4/9 of the reference,
and above 1 below that: 1.489 at a tenth, the gas of the parity workloads
with rho_ref = rho_l, at tau_a = 0.53 (lambda_g = 0.01).  The library's bound
rho_ref C_p,ref <= min rho C_p lies inside the stable range.  A mistake in the
rest equilibrium (e.g. the local rho C_p in place of the reference in its
rest term, the printed form that R4 replaces) moves these numbers.
"""

import numpy as np
import pytest

from oracle import oracle as O

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]


def growth(K, Eref, tau_a, nk=32):
    """Largest |eigenvalue| of one enthalpy LB step for heat capacity K =
    rho C_p and reference Eref = rho_ref C_p,ref, over a k-grid of [0, pi]^2."""
    A = O.heq(1.0, 0.0, K, Eref, 0.0, 0.0)      # d h^eq / d (rho H)
    B = O.heq(0.0, 1.0, K, Eref, 0.0, 0.0)      # d h^eq / d T
    E = np.outer(A + B / K, np.ones(9))          # h -> h^eq (T = rho H / K)
    tau_s = 1.0 / (2.0 - 1.0 / tau_a)
    P = np.zeros((9, 9))
    P[np.arange(9), OPP] = 1.0
    sym, anti = 0.5 * (np.eye(9) + P), 0.5 * (np.eye(9) - P)
    col = np.eye(9) - (anti / tau_a + sym / tau_s) @ (np.eye(9) - E)
    cx, cy = np.array(CX), np.array(CY)
    g = 0.0
    for kx in np.linspace(0.0, np.pi, nk):
        for ky in np.linspace(0.0, np.pi, nk):
            S = np.exp(-1j * (kx * cx + ky * cy))[:, None] * col
            g = max(g, float(np.abs(np.linalg.eigvals(S)).max()))
    return g


def test_equilibrium_at_rest_sums_to_the_enthalpy():
    h = O.heq(0.7, -0.3, 0.25, 1.0, 0.0, 0.0)
    assert abs(h.sum() - 0.7) < 1e-15
    # moving populations carry w_i rho_ref C_p,ref T, not the local capacity
    assert np.allclose(h[1:5], -0.3 / 9) and np.allclose(h[5:], -0.3 / 36)


def test_growth_factor_of_the_gas_with_the_liquid_reference():
    # gas of the parity workloads (rho_g C_p,g = 0.1) with rho_ref C_p,ref = 1
    g = growth(0.1, 1.0, 0.53, nk=48)
    assert abs(g - 1.4887) < 2e-3, g


@pytest.mark.parametrize("tau_a", [0.53, 0.8, 1.5])
def test_stable_exactly_above_the_rest_weight(tau_a):
    w0 = 4.0 / 9.0
    assert growth(w0 * 0.98, 1.0, tau_a) > 1.0 + 1e-4
    for ratio in (w0 * 1.02, 0.6, 1.0, 2.0, 10.0):
        assert growth(ratio, 1.0, tau_a) <= 1.0 + 1e-12, ratio
