"""Pin of the oracle's chemical potential against the free energy it derives
from (no GPU).

The paper gives the free-energy functional eq44 and states that mu_phi is
its variational derivative.  Here eq44 is written out term by term as
printed, on a periodic lattice, with every gradient product taken in the
lattice's own difference form

    grad a . grad b  ->  3 sum_{i=1..8} w_i (a(x + c_i) - a(x)) (b(x + c_i) - b(x)),

whose derivative with respect to b(y) is -(1/2) times the isotropic
Laplacian 6 sum_i w_i (a(y + c_i) - a(y)) of a (for a = b: -1 times).  The
derivative of that discrete functional with respect to phi at one node is
then exactly the oracle's mu_phi at that node, evaluated with the oracle's
own stencil Laplacians of phi, phi0 and f_s.  The discrete functional is a
polynomial of degree four in each phi(y), so the five-point central
difference used below is exact up to rounding.

Every term is switched on (phi0, f_s, cos(theta) and cos(psi) all nonzero,
with values of order one), so a dropped term, a wrong sign or a wrong
coefficient in any of the eight terms of mu_phi -- including the ice-wetting
terms in cos(psi) -- moves mu_phi by far more than the tolerance.
"""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WI = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def grad_dot(a, b):
    """Per-node lattice form of grad a . grad b (periodic)."""
    out = np.zeros_like(a)
    for i in range(1, 9):
        da = np.roll(a, (-CY[i], -CX[i]), axis=(0, 1)) - a
        db = np.roll(b, (-CY[i], -CX[i]), axis=(0, 1)) - b
        out += 3.0 * WI[i] * da * db
    return out


def free_energy(phi, phi0, fs, sigma, eps, cth, cpsi):
    """Eq44 as printed, summed over the lattice."""
    dens = (3 * sigma / (4 * eps)) * (1 - phi) ** 2 * (1 + phi) ** 2 \
        + (3 * eps * sigma / 16) * grad_dot(phi, phi) \
        + (9 * sigma / (2 * eps)) * phi0 ** 2 * phi ** 2 \
        + (3 * sigma * cth / eps) * phi0 * phi * (phi ** 2 + phi0 ** 2 - 1) \
        + (3 * eps * sigma * cth / 8) * grad_dot(phi0, phi) \
        + (9 * sigma / (2 * eps)) * fs ** 2 * phi ** 2 \
        + (3 * sigma * cpsi / eps) * fs * phi * (phi ** 2 + fs ** 2 - 1) \
        + (3 * eps * sigma * cpsi / 8) * grad_dot(fs, phi)
    return float(dens.sum())


@pytest.mark.parametrize("seed,cth,cpsi", [(0, 0.5, 0.5), (1, -0.3, 0.8), (2, 0.9, -0.6),
                                           (3, 0.0, 0.7)])
def test_mu_phi_is_the_derivative_of_eq44(oracle_mod, seed, cth, cpsi):
    rng = np.random.default_rng(seed)
    ny, nx = 7, 9
    phi = rng.uniform(-1.0, 1.0, (ny, nx))
    phi0 = rng.uniform(0.0, 0.7, (ny, nx))
    fs = rng.uniform(0.0, 0.7, (ny, nx))
    case = W.sessile_drop(nx=nx, ny=ny)
    sigma, eps = 0.7, 3.0
    case.mat.sigma, case.mat.eps, case.mat.cos_psi = sigma, eps, cpsi
    _, _, lphi = oracle_mod.stencil(phi, True, True)
    _, _, lphi0 = oracle_mod.stencil(phi0, True, True)
    _, _, lfs = oracle_mod.stencil(fs, True, True)
    d = 0.05
    worst = 0.0
    for (y, x) in [(0, 0), (3, 4), (6, 8), (2, 7), (5, 1)]:
        vals = []
        for m in (-2, -1, 1, 2):
            p = phi.copy()
            p[y, x] += m * d
            vals.append(free_energy(p, phi0, fs, sigma, eps, cth, cpsi))
        fd = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * d)
        mu = oracle_mod.chem_pot(case, phi[y, x], lphi[y, x], phi0[y, x], cth, lphi0[y, x],
                                 fs[y, x], lfs[y, x])
        worst = max(worst, abs(mu - fd))
        assert abs(mu - fd) <= 1e-11 * max(1.0, abs(fd)), (y, x, mu, fd)
    assert worst < 1e-11

