"""Seeded synthetic inputs for the three-dimensional (D3Q19) coupled step.

Input data only (geometry, initial fields, boundary settings), no method
arithmetic: both the FP64 oracle and the HIP path read what it returns.
Every 3D field is a C-contiguous float64 array of shape (nz, ny, nx); node
(x, y, z) is element [z, y, x].  Faces: 0 x-low, 1 x-high, 2 y-low, 3 y-high,
4 z-low, 5 z-high; walls sit half-way outside the first and last node.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

from .workloads import ADIABATIC, DIRICHLET, Material

XL, XH, YL, YH, ZL, ZH = range(6)


@dataclasses.dataclass
class Case3:
    name: str
    nx: int
    ny: int
    nz: int
    periodic: Sequence[bool]          # (x, y, z)
    thermal_bc: Sequence[int]         # per face
    wall_T: Sequence[float]           # per face (Dirichlet faces)
    phi0: np.ndarray
    cos_theta: np.ndarray
    phi: np.ndarray
    T: np.ndarray
    mat: Material
    substrate_fixed: bool = False
    T_substrate: float = -1.0
    steps: int = 0

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz


def _tanh(d, eps):
    return np.tanh(2.0 * d / eps)


def _grid(nx, ny, nz):
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    return x, y, z


def from_2d(case2, axis: str = "z", depth: int = 1, name: Optional[str] = None) -> Case3:
    """A 2D case extruded along one periodic axis: 2D (x, y) become
    (x, y) for axis "z", (x, z) for axis "y", (y, z) for axis "x"; the 2D walls
    (bottom, top, left, right) map to the faces of the 2D axes."""
    nx2, ny2 = case2.nx, case2.ny

    def ext(a):
        a = np.asarray(a, dtype=np.float64)
        if axis == "z":
            return np.broadcast_to(a[None, :, :], (depth, ny2, nx2)).copy()
        if axis == "y":
            return np.broadcast_to(a[:, None, :], (ny2, depth, nx2)).copy()
        return np.broadcast_to(a[:, :, None], (ny2, nx2, depth)).copy()

    wall_T = [0.0] * 6
    tbc = [ADIABATIC] * 6
    # 2D walls: 0 bottom (y-low), 1 top (y-high), 2 left (x-low), 3 right (x-high)
    if axis == "z":
        nx, ny, nz = nx2, ny2, depth
        face = {0: YL, 1: YH, 2: XL, 3: XH}
        periodic = (case2.periodic_x, case2.periodic_y, True)
    elif axis == "y":
        nx, ny, nz = nx2, depth, ny2
        face = {0: ZL, 1: ZH, 2: XL, 3: XH}
        periodic = (case2.periodic_x, True, case2.periodic_y)
    else:
        nx, ny, nz = depth, nx2, ny2
        face = {0: ZL, 1: ZH, 2: YL, 3: YH}
        periodic = (True, case2.periodic_x, case2.periodic_y)
    for w in range(4):
        prof = np.asarray(case2.wall_profile(w), dtype=np.float64)
        if case2.thermal_bc[w]:
            if prof.size and np.ptp(prof) > 0:
                raise ValueError("3D faces take one temperature each")
            tbc[face[w]] = DIRICHLET
            wall_T[face[w]] = float(prof[0]) if prof.size else 0.0
    return Case3(name or f"{case2.name}_3d{axis}", nx, ny, nz, periodic, tbc, wall_T,
                 ext(case2.phi0), ext(case2.cos_theta), ext(case2.phi), ext(case2.T),
                 case2.mat, case2.substrate_fixed, case2.T_substrate, case2.steps)


def sphere_drop(n: int = 48, radius: float = 12.0, mat: Optional[Material] = None,
                T: float = 1.0) -> Case3:
    """A drop in a periodic box, isothermal above the melting point (Laplace)."""
    mat = mat or Material()
    x, y, z = _grid(n, n, n)
    c = (n - 1) / 2.0
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    zero = np.zeros((n, n, n))
    return Case3(f"sphere_{n}", n, n, n, (True, True, True), [ADIABATIC] * 6, [0.0] * 6,
                 zero.copy(), zero.copy(), _tanh(radius - r, mat.eps), np.full((n, n, n), T), mat)


def sessile_drop3(nx: int = 64, ny: int = 64, nz: int = 48, radius: float = 16.0,
                  h_s: float = 6.0, theta: float = 75.0, T_wall: float = -1.0,
                  mat: Optional[Material] = None) -> Case3:
    """A hemispherical drop on a diffuse slab over a cold wall (z-low Dirichlet),
    periodic in x and y, adiabatic top."""
    mat = mat or Material()
    x, y, z = _grid(nx, ny, nz)
    phi0 = 0.5 + 0.5 * _tanh(h_s - z, mat.eps)
    r = np.sqrt((x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2 + (z - h_s) ** 2)
    phi = (1.0 - phi0) * _tanh(radius - r, mat.eps)
    cth = np.full((nz, ny, nx), math.cos(math.radians(theta)))
    tbc = [ADIABATIC] * 6
    tbc[ZL] = DIRICHLET
    wall_T = [0.0] * 6
    wall_T[ZL] = T_wall
    return Case3(f"sessile3_{nx}x{ny}x{nz}", nx, ny, nz, (True, True, False), tbc, wall_T,
                 phi0, cth, phi, np.zeros((nz, ny, nx)), mat)


def _rough_surface(nx, ny, rng, std, min_wavelength, max_wavelength, slope=-1.5, modes=48):
    """Sum of random Fourier modes (wavelengths between the bounds, amplitude
    ~ k^slope), periodic in y, scaled to the given standard deviation."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    h = np.zeros((ny, nx))
    for _ in range(modes):
        lam = math.exp(rng.uniform(math.log(min_wavelength), math.log(max_wavelength)))
        k = 2 * math.pi / lam
        ang = rng.uniform(0, 2 * math.pi)
        ky = round(k * math.sin(ang) * ny / (2 * math.pi)) * 2 * math.pi / ny
        kx = k * math.cos(ang)
        h += k ** slope * np.cos(kx * x + ky * y + rng.uniform(0, 2 * math.pi))
    return h * (std / max(h.std(), 1e-12))


def fracture(nx: int = 256, ny: int = 128, nz: int = 30, seed: int = 9,
             aperture: float = 14.0, roughness: float = 2.5, mismatch: float = 30.0,
             T_wall: float = -1.0, mat: Optional[Material] = None, steps: int = 20000) -> Case3:
    """Freezing in a rough fracture (the set-up of Sec. 4.5 with a synthetic
    fracture in place of the generated one): walls normal to x (x-low cold
    Dirichlet, x-high adiabatic), periodic in y and z.  The two fracture
    surfaces share their long wavelengths (above the mismatch length) and
    differ below it; roughness is their standard deviation.  A liquid column
    fills x < 0.75 nx with three gas bubbles of radii 0.075, 0.05 and 0.01 nx
    at (0.25, 0.25, 0.5), (0.5, 0.5, 0.5), (0.25, 0.75, 0.5) of the box;
    wettability varies in smooth patches between 60 and 120 degrees."""
    mat = mat or Material()
    rng = np.random.default_rng(seed)
    common = _rough_surface(nx, ny, rng, roughness, mismatch, 4.0 * ny)
    lo = common + _rough_surface(nx, ny, rng, 0.5 * roughness, 6.0, mismatch)
    hi = common + _rough_surface(nx, ny, rng, 0.5 * roughness, 6.0, mismatch)
    x, y, z = _grid(nx, ny, nz)
    zc = (nz - 1) / 2.0
    z_lo = (zc - aperture / 2.0 + lo)[None, :, :]
    z_hi = (zc + aperture / 2.0 + hi)[None, :, :]
    # signed distance into the solid along z (periodic z: the two walls meet)
    d = np.maximum(z_lo - z, z - z_hi)
    phi0 = 0.5 + 0.5 * _tanh(d, mat.eps)
    liquid = _tanh(0.75 * nx - x, mat.eps)
    for (cx, cy, cz), r in (((0.25, 0.25, 0.5), 0.075), ((0.5, 0.5, 0.5), 0.05),
                            ((0.25, 0.75, 0.5), 0.01)):
        rr = np.sqrt((x - cx * nx) ** 2 + (y - cy * ny) ** 2 + (z - cz * nz) ** 2)
        liquid = np.minimum(liquid, _tanh(rr - r * nx, mat.eps))
    phi = (1.0 - phi0) * liquid
    patch = _rough_surface(nx, ny, rng, 1.0, 20.0, 2.0 * ny, slope=0.0)
    theta = 90.0 + 30.0 * np.clip(patch / 2.0, -1.0, 1.0)
    cth = np.broadcast_to(np.cos(np.radians(theta))[None, :, :], (nz, ny, nx)).copy()
    tbc = [ADIABATIC] * 6
    tbc[XL] = DIRICHLET
    wall_T = [0.0] * 6
    wall_T[XL] = T_wall
    return Case3(f"fracture_{nx}x{ny}x{nz}", nx, ny, nz, (False, True, True), tbc, wall_T,
                 phi0, cth, phi, np.zeros((nz, ny, nx)), mat, steps=steps)
