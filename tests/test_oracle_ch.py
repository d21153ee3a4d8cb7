"""Pins of the Cahn-Hilliard smoothing oracle (no GPU).

* the discrete Laplacian's symbol: a Fourier mode is an eigenvector with the
  eigenvalue of the closed form 6 sum_i w_i (cos(k.c_i) - 1), written out
  per lattice from the shells (axes, diagonals), and the largest magnitude
  over the Brillouin zone is 16/3 on both lattices;
* the linear growth rate of a small mode around a uniform state: one Euler
  step multiplies its amplitude by 1 + dt M L(k) (A (3 c0^2 - 1) - kappa L(k))
  (unstable inside the spinodal, damped outside);
* exact conservation of sum c with walls and with wrap;
* the free energy never increases;
* the flat equilibrium has the model's interface profile tanh(2 d / eps):
  the exact continuum profile barely moves, and a sharp step relaxes onto it;
* a z-invariant 3D image gives the 2D result (the D3Q19 weights summed over
  equal in-plane velocities are the D2Q9 weights);
* mirror symmetry of the walls; the saturation of the uniform pore mixture.
"""

import math

import numpy as np
import pytest

from oracle import ch_oracle as CH
from paper_2510_18688_amd import workloads as W


def symbol(k, dim):
    c = [math.cos(v) for v in k]
    if dim == 2:
        a, b = c
        return 6.0 * ((2.0 / 9.0) * (a + b - 2.0) + (1.0 / 9.0) * (a * b - 1.0))
    a, b, g = c
    return 6.0 * ((1.0 / 9.0) * (a + b + g - 3.0) + (1.0 / 9.0) * (a * b + b * g + g * a - 3.0))


@pytest.mark.parametrize("dim, n, modes", [(2, (12, 10), [(1, 0), (2, 3), (6, 5), (5, 1)]),
                                           (3, (8, 6, 10), [(1, 0, 0), (2, 3, 1), (4, 3, 5), (0, 1, 4)])])
def test_laplacian_symbol(dim, n, modes):
    grids = np.meshgrid(*[np.arange(v) for v in n[::-1]], indexing="ij")[::-1]   # x, y[, z]
    for m in modes:
        k = [2 * math.pi * m[a] / n[a] for a in range(dim)]
        X = np.cos(sum(k[a] * grids[a] for a in range(dim)) + 0.3)
        L = CH.laplacian(X, [True] * dim)
        assert np.abs(L - symbol(k, dim) * X).max() < 1e-12, m


def test_symbol_extremes():
    pts = np.linspace(-math.pi, math.pi, 41)
    m2 = min(symbol((a, b), 2) for a in pts for b in pts)
    m3 = min(symbol((a, b, c), 3) for a in pts for b in pts for c in pts)
    assert abs(m2 + 16 / 3) < 1e-12 and abs(m3 + 16 / 3) < 1e-12


@pytest.mark.parametrize("c0", [0.0, 0.3, 0.9])
def test_linear_growth_rate(c0):
    n = (16, 12)
    A, kappa, M, dt = 1.0, 2.0, 1.0, 0.02
    y, x = np.mgrid[0:n[1], 0:n[0]].astype(float)
    delta = 1e-5
    for m in [(1, 0), (1, 1), (3, 2), (8, 6)]:
        k = (2 * math.pi * m[0] / n[0], 2 * math.pi * m[1] / n[1])
        mode = np.cos(k[0] * x + k[1] * y)
        c1 = CH.ch_step(c0 + delta * mode, (True, True), A, kappa, M, dt)
        amp = float(np.sum((c1 - c1.mean()) * mode) / np.sum(mode * mode)) / delta
        L = symbol(k, 2)
        expect = 1.0 + dt * M * L * (A * (3 * c0 * c0 - 1.0) - kappa * L)
        assert abs(amp - expect) < 1e-8, (m, amp, expect)


@pytest.mark.parametrize("shape, periodic", [((40, 56), (False, False)), ((40, 56), (True, False)),
                                             ((12, 14, 16), (False, True, False))])
def test_mass_conservation(shape, periodic):
    img = W.sandpack_image(shape, seed=5, r_median=3.0, periodic=periodic)
    c0 = 2.0 * img - 1.0
    _, c = CH.smooth(img, periodic, 150, return_c=True)
    assert abs(c.sum() - c0.sum()) < 1e-10 * c.size


def test_free_energy_decreases():
    img = W.sandpack_image((48, 48), seed=2, r_median=4.0)
    per = (False, False)
    c = 2.0 * img - 1.0
    kap = CH.kappa_for(4.0)
    F = CH.free_energy(c, per, 1.0, kap)
    for _ in range(200):
        c = CH.ch_step(c, per, 1.0, kap, 1.0, 0.02)
        F1 = CH.free_energy(c, per, 1.0, kap)
        assert F1 <= F + 1e-12 * abs(F)
        F = F1


def test_flat_equilibrium_is_the_model_profile():
    """Two flat interfaces 48 nodes apart: the continuum profile tanh(2d/eps)
    is stationary up to the lattice's discretisation (1.3e-2 with the width
    eps/(2 sqrt 2) = 1.4 nodes), and a sharp step relaxes onto it (1.6e-2);
    a width 20 % off misses it by 6.7e-2, kappa doubled or halved by more
    than 0.13."""
    eps, nx = 4.0, 96
    x = np.arange(nx, dtype=float) + 0.5
    d = np.minimum(x - 24.0, 72.0 - x)
    exact = np.tanh(2.0 * d / eps)[None, :].repeat(4, axis=0)
    c = exact.copy()
    kap = CH.kappa_for(eps)
    for _ in range(2000):
        c = CH.ch_step(c, (True, True), 1.0, kap, 1.0, 0.02)
    assert np.abs(c - exact).max() < 0.02
    step = (d > 0).astype(np.uint8)[None, :].repeat(4, axis=0)
    _, cs = CH.smooth(step, (True, True), 2000, eps=eps, return_c=True)
    assert np.abs(cs - exact).max() < 0.025
    for f in (math.sqrt(2), 1 / math.sqrt(2), 1.2):
        _, cw = CH.smooth(step, (True, True), 2000, eps=eps * f, return_c=True)
        assert np.abs(cw - exact).max() > 0.05, f


def test_3d_extrusion_equals_2d():
    img = W.sandpack_image((30, 34), seed=3, r_median=4.0)
    p2 = CH.smooth(img, (False, True), 60)
    img3 = np.repeat(img[None, :, :], 3, axis=0)
    p3 = CH.smooth(img3, (False, True, True), 60)
    for z in range(3):
        assert np.abs(p3[z] - p2).max() < 1e-13


def test_mirror_symmetry_of_walls():
    img = W.sandpack_image((30, 17), seed=4, r_median=4.0)
    img = np.maximum(img, img[:, ::-1])
    p = CH.smooth(img, (False, False), 100)
    assert np.abs(p - p[:, ::-1]).max() < 1e-13
    img = np.maximum(img, img[::-1, :])
    p = CH.smooth(img, (False, False), 100)
    assert np.abs(p - p[::-1, :]).max() < 1e-13


def test_smoothing_keeps_the_grains_and_bounds():
    img = W.sandpack_image((64, 64), seed=8, r_median=6.0)
    p = CH.smooth(img, (False, False), 500)
    assert p.min() >= 0.0 and p.max() <= 1.0
    # the indicator stays on the image's side of 1/2 at all but a few nodes
    # (3.8 % at t = 10: the equation rounds grain corners and necks, and a
    # longer evolution coarsens the pack further)
    assert np.mean(np.abs(p - img) > 0.5) < 0.05


def test_saturation_of_the_uniform_mixture():
    img = W.sandpack_image((40, 60), seed=1, r_median=4.0)
    phi0 = CH.smooth(img, (False, False), 100)
    for S in (0.2, 0.32, 0.7):
        case = W.unsaturated_medium(phi0, S_w=S)
        assert abs(CH.saturation(phi0, case.phi) - S) < 1e-14
