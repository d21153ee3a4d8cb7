"""Seeded synthetic inputs for the coupled freezing step.

This module only builds *input data*: material constants, the diffuse solid
label phi0, the wettability field cos(theta), the initial order parameter and
temperature, and the wall-temperature profiles.  It holds none of the method's
arithmetic (no equilibria, no enthalpy map, no relaxation times), so both the
FP64 oracle and the HIP path may read what it returns.

Array convention: every 2D field is a C-contiguous float64 array of shape
(ny, nx); node (x, y) is element [y, x].  Walls, where present, sit half-way
between nodes, at y = -1/2 and y = ny - 1/2 (x = -1/2 and x = nx - 1/2).

Geometry and initial profiles follow the paper's tanh set-ups: the slab form
of phi0 and phi in Sec. 4.2 (eq_initial) and the curved-substrate form in
Sec. 4.4 (initialc), with interface width W = epsilon and profile
tanh(2 d / epsilon).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

# wall indices used by every profile dictionary below
BOTTOM, TOP, LEFT, RIGHT = 0, 1, 2, 3
ADIABATIC, DIRICHLET = 0, 1


@dataclasses.dataclass
class Material:
    """Lattice-unit material constants (Delta x = Delta t = 1).

    Defaults are the paper's lattice values where it gives them (sigma,
    mobility, liquid viscosity, epsilon: Sec. 4.2 and Sec. 4.4) and the
    stated property ratios of the droplet workloads otherwise: gas/liquid
    density 0.1, solid/liquid density 0.9, gas/liquid viscosity 0.1,
    equal heat capacities, Stefan number 1 at T_w = -1.
    """

    rho_l: float = 1.0
    rho_g: float = 0.1
    rho_s: float = 0.9
    mu_l: float = 0.1
    mu_g: float = 0.01
    mu_s: float = 0.1
    lam_l: float = 0.1
    lam_g: float = 0.01
    lam_s: float = 0.1
    cp_l: float = 1.0
    cp_g: float = 1.0
    cp_s: float = 1.0
    latent: float = 1.0
    T_m: float = 0.0
    sigma: float = 1e-3
    eps: float = 4.0
    mobility: float = 0.1
    cos_psi: float = 0.0
    rho_ref: float = 0.1
    pcm_floor: float = 0.01
    latch_fs: int = 1
    h_src_tau_a: int = 0
    # div u of the phase-field source and recovery: 0 the divergence of the
    # previous step's velocity (the flow's own), 1 the model's mass source mdot
    phi_src_mdot: int = 0
    # flow and phase-field collisions: 0 BGK (Sec. 3.1, 3.2), 1 MRT with the
    # bulk rate s_b (density, energy and energy-square moments of f), the
    # energy-flux rate s_q of f and the rate s_g of the moments of g above
    # first order; 0 stands for the BGK rate (1/tau_f, 1/tau_g)
    mrt: int = 0
    s_b: float = 0.0
    s_q: float = 0.0
    s_g: float = 0.0
    # body force G = rho g (gravitational acceleration g) and the velocity
    # u_s of the solid phase in the drag (Sec. 3.1); z components for 3D
    g_x: float = 0.0
    g_y: float = 0.0
    g_z: float = 0.0
    us_x: float = 0.0
    us_y: float = 0.0
    us_z: float = 0.0

    def as_dict(self) -> Dict[str, float]:
        return dataclasses.asdict(self)


@dataclasses.dataclass
class Case:
    """One lattice problem: sizes, boundary types, fields and material."""

    name: str
    nx: int
    ny: int
    periodic_x: bool
    periodic_y: bool
    thermal_bc: List[int]            # per wall: ADIABATIC or DIRICHLET
    wall_T: Dict[int, np.ndarray]    # per Dirichlet wall: profile along it
    phi0: np.ndarray
    cos_theta: np.ndarray
    phi: np.ndarray
    T: np.ndarray
    mat: Material
    substrate_fixed: bool = False    # nodes with phi0 >= 1/2 held at T_substrate
    T_substrate: float = 0.0
    steps: int = 0
    # per-node isothermal region: held temperature of each node, NaN where
    # the node is free (replaces the substrate_fixed rule when given)
    T_hold: Optional[np.ndarray] = None

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def wall_profile(self, wall: int) -> np.ndarray:
        n = self.nx if wall in (BOTTOM, TOP) else self.ny
        if wall in self.wall_T:
            return np.ascontiguousarray(self.wall_T[wall], dtype=np.float64)
        return np.zeros(n, dtype=np.float64)


def _grid(nx: int, ny: int):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return x, y


def _tanh_profile(d: np.ndarray, eps: float) -> np.ndarray:
    return np.tanh(2.0 * d / eps)


def slab_phi0(nx: int, ny: int, h_s: float, eps: float) -> np.ndarray:
    """Pre-existing solid slab below y = h_s (eq_initial, Sec. 4.2)."""
    _, y = _grid(nx, ny)
    return 0.5 + 0.5 * _tanh_profile(h_s - y, eps)


def sessile_drop(nx: int = 128, ny: int = 96, radius: float = 30.0,
                 T_wall: float = -1.0, steps: int = 5000,
                 mat: Optional[Material] = None) -> Case:
    """Sessile drop on a bare flat cold wall (90 degrees), 128 x 96.

    Periodic in x; bounce-back walls in y; bottom wall at T_wall, top wall
    adiabatic.  Drop centred on the bottom wall, at (nx/2, -1/2).
    """
    mat = mat or Material()
    x, y = _grid(nx, ny)
    r = np.hypot(x - nx / 2.0, y + 0.5)
    phi = _tanh_profile(radius - r, mat.eps)
    zeros = np.zeros((ny, nx))
    return Case("sessile_flat_128x96", nx, ny, True, False,
                [DIRICHLET, ADIABATIC, ADIABATIC, ADIABATIC],
                {BOTTOM: np.full(nx, T_wall)}, zeros.copy(), zeros.copy(),
                phi, zeros.copy(), mat, steps=steps)


def curved_substrate(n: int = 2048, R_s: float = 400.0, R_0: float = 300.0,
                     theta_deg: float = 60.0, T_sub: float = -1.0,
                     steps: int = 20000, mat: Optional[Material] = None) -> Case:
    """Drop on a cold cylinder (initialc set-up, Sec. 4.4), n x n lattice.

    Cylinder centre (n/2, n/4), radius R_s; drop centre on its top,
    (n/2, n/4 + R_s), radius R_0.  Periodic x, adiabatic walls in y; solid
    nodes (phi0 >= 1/2) held at T_sub.
    """
    mat = mat or Material()
    x, y = _grid(n, n)
    rc = np.hypot(x - n / 2.0, y - n / 4.0)
    phi0 = 0.5 + 0.5 * _tanh_profile(R_s - rc, mat.eps)
    rd = np.hypot(x - n / 2.0, y - n / 4.0 - R_s)
    phi = (1.0 - phi0) * _tanh_profile(R_0 - rd, mat.eps)
    cth = np.full((n, n), math.cos(math.radians(theta_deg)))
    T = np.where(phi0 >= 0.5, T_sub, 0.0)
    return Case(f"curved_substrate_{n}x{n}", n, n, True, False,
                [ADIABATIC, ADIABATIC, ADIABATIC, ADIABATIC], {},
                phi0, cth, phi, T, mat, substrate_fixed=True,
                T_substrate=T_sub, steps=steps)


def porous_grains(nx: int, ny: int, seed: int = 3, porosity: float = 0.6,
                  rmin: float = 20.0, rmax: float = 60.0, gap: float = 8.0,
                  max_tries: int = 2_000_000):
    """Random sequential addition of non-overlapping disks.

    Radii uniform in [rmin, rmax]; centres uniform with clearance r + gap to
    the walls and r_a + r_b + gap between grains; stops once the grain area
    reaches (1 - porosity) of the box.
    """
    rng = np.random.default_rng(seed)
    target = (1.0 - porosity) * nx * ny
    cx: List[float] = []
    cy: List[float] = []
    rr: List[float] = []
    area = 0.0
    tries = 0
    # coarse bucket grid for the overlap test
    cell = 2 * rmax + gap
    buckets: Dict[tuple, List[int]] = {}
    while area < target and tries < max_tries:
        tries += 1
        r = rng.uniform(rmin, rmax)
        px = rng.uniform(r + gap, nx - r - gap)
        py = rng.uniform(r + gap, ny - r - gap)
        bx, by = int(px // cell), int(py // cell)
        ok = True
        for ix in (bx - 1, bx, bx + 1):
            for iy in (by - 1, by, by + 1):
                for k in buckets.get((ix, iy), ()):
                    if math.hypot(px - cx[k], py - cy[k]) < r + rr[k] + gap:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        buckets.setdefault((bx, by), []).append(len(rr))
        cx.append(px)
        cy.append(py)
        rr.append(r)
        area += math.pi * r * r
    return np.array(cx), np.array(cy), np.array(rr)


def porous_medium(nx: int = 4096, ny: int = 2048, seed: int = 3,
                  theta_deg: float = 45.0, T_cold: float = -1.0,
                  T_hot: float = 0.0, steps: int = 50000,
                  mat: Optional[Material] = None, rmin: float = 20.0,
                  rmax: float = 60.0, porosity: float = 0.6) -> Case:
    """Porous medium of random grains, left half liquid, right half gas.

    Walls on all sides; left wall at T_cold, right wall at T_hot, top and
    bottom adiabatic (the porous set-up of Sec. 4.6).
    """
    mat = mat or Material()
    cx, cy, rr = porous_grains(nx, ny, seed=seed, porosity=porosity, rmin=rmin, rmax=rmax)
    phi0 = np.zeros((ny, nx))
    pad = int(3 * mat.eps)
    for px, py, r in zip(cx, cy, rr):
        x0 = max(0, int(px - r - pad)); x1 = min(nx, int(px + r + pad) + 1)
        y0 = max(0, int(py - r - pad)); y1 = min(ny, int(py + r + pad) + 1)
        yy, xx = np.mgrid[y0:y1, x0:x1].astype(np.float64)
        d = np.hypot(xx - px, yy - py)
        lab = 0.5 + 0.5 * _tanh_profile(r - d, mat.eps)
        np.maximum(phi0[y0:y1, x0:x1], lab, out=phi0[y0:y1, x0:x1])
    x, _ = _grid(nx, ny)
    phi = (1.0 - phi0) * _tanh_profile(nx / 2.0 - x, mat.eps)
    cth = np.full((ny, nx), math.cos(math.radians(theta_deg)))
    return Case(f"porous_{nx}x{ny}", nx, ny, False, False,
                [ADIABATIC, ADIABATIC, DIRICHLET, DIRICHLET],
                {LEFT: np.full(ny, T_cold), RIGHT: np.full(ny, T_hot)},
                phi0, cth, phi, np.zeros((ny, nx)), mat, steps=steps)


def slab_drop(nx: int, ny: int, radius: float, theta, T_wall,
              h_s: float = 10.0, steps: int = 0,
              mat: Optional[Material] = None, name: str = "slab_drop") -> Case:
    """Drop resting on a diffuse solid slab of height h_s above a cold wall.

    theta: contact angle in degrees, scalar or per-column array (nx,).
    T_wall: bottom-wall temperature, scalar or per-column array (nx,).
    Periodic in x; walls in y; bottom Dirichlet, top adiabatic.
    """
    mat = mat or Material()
    x, y = _grid(nx, ny)
    phi0 = slab_phi0(nx, ny, h_s, mat.eps)
    r = np.hypot(x - nx / 2.0, y - h_s)
    phi = (1.0 - phi0) * _tanh_profile(radius - r, mat.eps)
    th = np.broadcast_to(np.asarray(theta, dtype=np.float64), (nx,))
    cth = np.broadcast_to(np.cos(np.radians(th))[None, :], (ny, nx)).copy()
    Tw = np.broadcast_to(np.asarray(T_wall, dtype=np.float64), (nx,)).copy()
    return Case(name, nx, ny, True, False,
                [DIRICHLET, ADIABATIC, ADIABATIC, ADIABATIC],
                {BOTTOM: Tw}, phi0, cth, phi, np.zeros((ny, nx)), mat,
                steps=steps)


def batch_instances(count: int = 64, seed: int = 4, lo: int = 64,
                    hi: int = 512) -> List[Case]:
    """Uneven droplet-freezing instances for one batched launch.

    Sides log-uniform in [lo, hi] (redrawn if equal), nx >= ny; radius 0.3 x
    the shorter side; contact angle uniform in [30, 150] degrees; wall
    temperature uniform in [-2, -0.5].
    """
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(count):
        while True:
            a, b = np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), 2)))
            if a != b:
                break
        nx, ny = int(max(a, b)), int(min(a, b))
        theta = float(rng.uniform(30.0, 150.0))
        Tw = float(rng.uniform(-2.0, -0.5))
        cases.append(slab_drop(nx, ny, round(0.3 * ny), theta, Tw,
                               name=f"batch{k}_{nx}x{ny}"))
    return cases


def fourier_modes(n: int, rng: np.random.Generator, modes: int = 4) -> np.ndarray:
    """Sum of random periodic Fourier modes on n points, scaled to max |s| = 1."""
    x = np.arange(n, dtype=np.float64)
    s = np.zeros(n)
    for _ in range(modes):
        k = int(rng.integers(1, 6))
        amp = rng.normal()
        ph = rng.uniform(0.0, 2.0 * math.pi)
        s += amp * np.cos(2.0 * math.pi * k * x / n + ph)
    return s / np.max(np.abs(s))


def adjoint_case(n: int = 256, steps: int = 2000, radius: float = 77.0):
    """Flat-wall drop for the gradient workload and its seeded target controls.

    Returns (case, theta_target_deg, Tw_target) where the target controls are
    90 deg + 15 deg s1(x) and -1 + 0.25 s2(x).
    """
    case = slab_drop(n, n, radius, 90.0, -1.0, steps=steps, name=f"adjoint_{n}x{n}")
    case.mat.phi_src_mdot = 1   # the phase-field source the reverse sweep differentiates
    rng = np.random.default_rng(5)
    s1 = fourier_modes(n, rng)
    s2 = fourier_modes(n, rng)
    return case, 90.0 + 15.0 * s1, -1.0 + 0.25 * s2


def small_freezing_case(nx: int = 32, ny: int = 24, h_s: float = 3.0, radius: float = 8.0,
                        T_wall: float = -1.5, seed: int = 1) -> Case:
    """A small drop on a thin diffuse slab over a cold wall: the cold front
    reaches the drop within tens of steps, so the final ice fraction depends
    on both the wettability and the wall temperature.  Contact angles
    75 +- 10 degrees and wall temperatures T_wall +- 0.2, drawn per column."""
    case = slab_drop(nx, ny, radius, 75.0, T_wall, h_s=h_s, name=f"small_freezing_{nx}x{ny}")
    case.mat.phi_src_mdot = 1   # the phase-field source the reverse sweep differentiates
    rng = np.random.default_rng(seed)
    th = 75.0 + 10.0 * rng.uniform(-1, 1, nx)
    case.cos_theta = np.broadcast_to(np.cos(np.radians(th))[None, :], (ny, nx)).copy()
    case.wall_T = {BOTTOM: T_wall + 0.2 * rng.uniform(-1, 1, nx)}
    return case


WORKLOADS = {
    "sessile_flat_128x96": lambda: sessile_drop(),
    "curved_substrate_2048x2048": lambda: curved_substrate(),
    "porous_4096x2048": lambda: porous_medium(),
}


def sandpack_image(shape, porosity: float = 0.3585, seed: int = 12, r_median: float = 8.0,
                   sigma_log: float = 0.45, r_min: float = 2.5, periodic=(False, False, False),
                   max_grains: int = 2_000_000) -> np.ndarray:
    """Binary image of a poorly sorted, unconsolidated grain pack (1 = solid):
    overlapping disks (2D shape (ny, nx)) or spheres (3D shape (nz, ny, nx))
    with log-normal radii (median r_median, log standard deviation
    sigma_log, floored at r_min), centres uniform in the box, added until the
    pore fraction falls to `porosity`.  Grains wrap across periodic axes."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in shape)
    dim = len(shape)
    img = np.zeros(shape, dtype=np.uint8)
    total = img.size
    solid = 0
    target = (1.0 - porosity) * total
    axes_n = shape[::-1]            # (nx, ny[, nz])
    for _ in range(max_grains):
        if solid >= target:
            break
        r = max(r_min, r_median * math.exp(sigma_log * rng.standard_normal()))
        ctr = [rng.uniform(0.0, n) for n in axes_n]
        idx, off = [], []
        for a in range(dim):
            lo, hi = int(math.floor(ctr[a] - r)), int(math.ceil(ctr[a] + r)) + 1
            i = np.arange(lo, hi)
            if periodic[a]:
                sel = np.ones(i.size, dtype=bool)
                ii = np.mod(i, axes_n[a])
            else:
                sel = (i >= 0) & (i < axes_n[a])
                ii = i[sel]
            idx.append(ii)
            off.append((i[sel] + 0.5 - ctr[a]) ** 2)
        d2 = off[0][None, :] + off[1][:, None] if dim == 2 else (
            off[0][None, None, :] + off[1][None, :, None] + off[2][:, None, None])
        inside = d2 <= r * r
        sub = img[np.ix_(*idx[::-1])]
        new = int(np.count_nonzero(inside & (sub == 0)))
        if new:
            sub = sub | inside.astype(np.uint8)
            img[np.ix_(*idx[::-1])] = sub
            solid += new
    return img


def unsaturated_medium(phi0: np.ndarray, S_w: float = 0.32, theta_deg: float = 60.0,
                       T0: float = 0.5, steps: int = 0, mat: Optional[Material] = None,
                       name: str = "unsaturated", gravity=(0.0, 0.0)) -> Case:
    """The unsaturated porous set-up of Sec. 4.6 on a 2D solid indicator phi0
    (ny, nx): the pores hold phi = (1 - phi0) phi_i with phi_i = 2 S_w - 1
    (a uniform mixture whose liquid share of the pore volume is S_w), at a
    uniform T0 above melting; walls on all sides, the x walls Dirichlet at
    T0 for the phase-separation stage (`wall_T_freezing` gives the cold and
    warm x walls of the freezing stage), the y walls adiabatic.  `gravity`:
    the acceleration (x, y) of the body force rho g, which with cohesion and
    adhesion sets where the liquid settles."""
    mat = dataclasses.replace(mat or Material(), g_x=float(gravity[0]), g_y=float(gravity[1]))
    ny, nx = phi0.shape
    phi_i = 2.0 * S_w - 1.0
    phi = (1.0 - phi0) * phi_i
    cth = np.full((ny, nx), math.cos(math.radians(theta_deg)))
    return Case(f"{name}_{nx}x{ny}_Sw{S_w:g}_th{theta_deg:g}", nx, ny, False, False,
                [ADIABATIC, ADIABATIC, DIRICHLET, DIRICHLET],
                {LEFT: np.full(ny, T0), RIGHT: np.full(ny, T0)},
                np.asarray(phi0, dtype=np.float64), cth, phi, np.full((ny, nx), T0), mat,
                steps=steps)


def wall_T_freezing(case: Case, T_cold: float = -1.0, T_hot: float = 0.5) -> Dict[int, np.ndarray]:
    """Wall temperatures of the freezing stage of `unsaturated_medium`."""
    return {LEFT: np.full(case.ny, T_cold), RIGHT: np.full(case.ny, T_hot)}
