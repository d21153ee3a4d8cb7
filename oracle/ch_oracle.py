"""Cahn-Hilliard smoothing of a binary solid image into the solid indicator
phi0 (plain numpy, FP64).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).

Sec. 4.6 smooths the sharp sandpack image by a finite-time evolution of a
standard Cahn-Hilliard equation before the LB run, without giving the
equation's form, parameters or discretisation.  Reading used here (the same
in the GPU path):

  * order parameter c = 2 s - 1 from the binary image s (1 in the solid);
  * the standard equation dc/dt = M lap(mu), mu = A (c^3 - c) - kappa lap(c),
    with kappa = A eps^2 / 8: its flat equilibrium profile is
    c = tanh(2 d / eps), so the smoothed indicator has the interface profile
    phi0 = 1/2 + 1/2 tanh(2 d / eps) that the model prescribes for the solid
    (Sec. 2) and the same width eps as the fluid-fluid interfaces;
  * lap is the lattice's isotropic Laplacian, 6 sum_i w_i (X(x + c_i) - X(x))
    with the D2Q9 weights for a 2D image and the D3Q19 weights for a 3D one
    (Sec. 3.1), periodic wrap or the mirror ghost (the first node repeated
    beyond a wall) per axis, as for the model's own stencils;
  * explicit Euler steps of size dt; phi0 = clamp((1 + c) / 2, 0, 1) at the
    end.

Arrays are [ny, nx] (2D) or [nz, ny, nx] (3D).
"""

from __future__ import annotations

import itertools
from typing import Sequence

import numpy as np


def velocities(dim: int):
    """Non-rest velocities and weights: D2Q9 (1/9 axes, 1/36 diagonals) or
    D3Q19 (1/18 axes, 1/36 face diagonals)."""
    out = []
    for c in itertools.product((-1, 0, 1), repeat=dim):
        n = sum(abs(v) for v in c)
        if n == 0 or n > 2:
            continue
        if dim == 2:
            w = 1.0 / 9.0 if n == 1 else 1.0 / 36.0
        else:
            w = 1.0 / 18.0 if n == 1 else 1.0 / 36.0
        out.append((c, w))
    return out


def neighbour_index(n: int, shift: int, periodic: bool) -> np.ndarray:
    """Index of x + shift along one axis: wrapped, or clamped to the first
    and last node (mirror ghost)."""
    i = np.arange(n) + shift
    return np.mod(i, n) if periodic else np.clip(i, 0, n - 1)


def laplacian(X: np.ndarray, periodic: Sequence[bool]) -> np.ndarray:
    """6 sum_i w_i (X(x + c_i) - X(x)); `periodic` per axis in (x, y[, z])
    order, X indexed [..., y, x]."""
    dim = X.ndim
    out = np.zeros_like(X)
    for c, w in velocities(dim):
        # c is (cx, cy[, cz]); array axes are reversed
        idx = [neighbour_index(X.shape[dim - 1 - a], c[a], bool(periodic[a])) for a in range(dim)]
        out += w * (X[np.ix_(*idx[::-1])] - X)
    return 6.0 * out


def chemical_potential(c: np.ndarray, periodic, A: float, kappa: float) -> np.ndarray:
    return A * (c ** 3 - c) - kappa * laplacian(c, periodic)


def ch_step(c: np.ndarray, periodic, A: float, kappa: float, mobility: float,
            dt: float) -> np.ndarray:
    """One explicit Euler step of dc/dt = M lap(mu)."""
    mu = chemical_potential(c, periodic, A, kappa)
    return c + dt * mobility * laplacian(mu, periodic)


def free_energy(c: np.ndarray, periodic, A: float, kappa: float) -> float:
    """Discrete Ginzburg-Landau energy sum A/4 (c^2 - 1)^2 - kappa/2 c lap(c),
    the Lyapunov functional of the equation (summation by parts of the
    gradient term, exact for the symmetric lattice Laplacian)."""
    return float(np.sum(0.25 * A * (c * c - 1.0) ** 2 - 0.5 * kappa * c * laplacian(c, periodic)))


def kappa_for(eps: float, A: float = 1.0) -> float:
    """kappa whose flat equilibrium is tanh(2 d / eps)."""
    return A * eps * eps / 8.0


def smooth(solid: np.ndarray, periodic, iterations: int, eps: float = 4.0, A: float = 1.0,
           mobility: float = 1.0, dt: float = 0.02, return_c: bool = False):
    """phi0 of a binary image after `iterations` Euler steps."""
    c = 2.0 * (np.asarray(solid) != 0).astype(np.float64) - 1.0
    kappa = kappa_for(eps, A)
    for _ in range(iterations):
        c = ch_step(c, periodic, A, kappa, mobility, dt)
    phi0 = np.clip(0.5 * (1.0 + c), 0.0, 1.0)
    return (phi0, c) if return_c else phi0


def saturation(phi0: np.ndarray, phi: np.ndarray) -> float:
    """Water saturation: liquid volume over pore volume, with the liquid
    volume sum (1 - phi0 + phi) / 2 (the phase-change-material fraction C of
    the model, no ice) and the pore volume sum (1 - phi0)."""
    return float(np.sum(0.5 * (1.0 - phi0 + phi)) / np.sum(1.0 - phi0))
