"""ctypes front end of the FP64 C oracle (test infrastructure only).

The C source, lbf_oracle.c, is a plain transcription of the coupled step of
Sec. 3 of the paper; this module only builds it, marshals arrays and names the
outputs.  Only tests, the smoke check and the benchmark's CPU baseline may use
it.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbf_oracle.c")
LIB = os.path.join(HERE, "liblbf_oracle.so")

FIELDS = ["phi", "T", "fl", "fs", "ux", "uy", "p", "rhoH", "mu", "C", "chi", "rho", "phihat"]
# lagged fields of the state: f_s, Q = rho C_p T mdot, (phi u)_x, (phi u)_y,
# p and u_x, u_y of the previous step
NLAG = 7
REDS = ["sum_g", "sum_h", "sum_fs", "sum_liq", "umax", "nonfinite",
        "src_phi", "src_heat", "wall_flux", "reset", "step"]


class OrcParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("periodic_x", C.c_int32),
                ("periodic_y", C.c_int32), ("thermal_bc", C.c_int32 * 4),
                ("latch_fs", C.c_int32), ("h_src_tau_a", C.c_int32),
                ("substrate_fixed", C.c_int32), ("pad_", C.c_int32)] + [
        (k, C.c_double) for k in (
            "rho_l", "rho_g", "rho_s", "mu_l", "mu_g", "mu_s", "lam_l", "lam_g", "lam_s",
            "cp_l", "cp_g", "cp_s", "latent", "T_m", "sigma", "eps", "mobility",
            "cos_psi", "rho_ref", "T_substrate", "pcm_floor")] + [
        ("mrt", C.c_int32), ("pad2_", C.c_int32), ("phi_src_mdot", C.c_int32),
        ("pad3_", C.c_int32), ("s_b", C.c_double), ("s_q", C.c_double),
        ("s_g", C.c_double), ("grav", C.c_double * 2), ("u_solid", C.c_double * 2)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcParams)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_init.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_fields.argtypes = [C.c_void_p, dp]
        L.orc_reduce.argtypes = [C.c_void_p, dp]
        L.orc_set_wall_T.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_set_cos_theta.argtypes = [C.c_void_p, dp]
        L.orc_set_isothermal.argtypes = [C.c_void_p, dp]
        L.orc_get_state.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_set_state.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_feq.argtypes = [C.c_double] * 4 + [dp]
        L.orc_mrt_matrix.argtypes = [dp]
        L.orc_invert9.argtypes = [dp, dp]
        L.orc_geq.argtypes = [C.c_double] * 4 + [dp]
        L.orc_heq.argtypes = [C.c_double] * 6 + [dp]
        L.orc_forcing.argtypes = [C.c_double] * 9 + [dp]
        L.orc_hmap.argtypes = [C.POINTER(OrcParams)] + [C.c_double] * 4 + [dp]
        L.orc_stencil.argtypes = [C.c_int] * 4 + [dp, dp, dp, dp]
        L.orc_chem_pot.restype = C.c_double
        L.orc_chem_pot.argtypes = [C.POINTER(OrcParams)] + [C.c_double] * 7
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_max_threads.restype = C.c_int
        L.orc_set_store_f32.argtypes = [C.c_void_p, C.c_int]
        L.orc_step_count.restype = C.c_long
        L.orc_step_count.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(case) -> OrcParams:
    p = OrcParams()
    p.nx, p.ny = case.nx, case.ny
    p.periodic_x, p.periodic_y = int(case.periodic_x), int(case.periodic_y)
    for w in range(4):
        p.thermal_bc[w] = int(case.thermal_bc[w])
    m = case.mat
    p.latch_fs, p.h_src_tau_a = int(m.latch_fs), int(m.h_src_tau_a)
    p.substrate_fixed = int(case.substrate_fixed)
    for k in ("rho_l", "rho_g", "rho_s", "mu_l", "mu_g", "mu_s", "lam_l", "lam_g",
              "lam_s", "cp_l", "cp_g", "cp_s", "latent", "T_m", "sigma", "eps",
              "mobility", "cos_psi", "rho_ref", "pcm_floor"):
        setattr(p, k, float(getattr(m, k)))
    p.T_substrate = float(case.T_substrate)
    p.mrt = int(getattr(m, "mrt", 0))
    p.phi_src_mdot = int(getattr(m, "phi_src_mdot", 0))
    p.s_b, p.s_q = float(getattr(m, "s_b", 0.0)), float(getattr(m, "s_q", 0.0))
    p.s_g = float(getattr(m, "s_g", 0.0))
    p.grav[0], p.grav[1] = float(m.g_x), float(m.g_y)
    p.u_solid[0], p.u_solid[1] = float(m.us_x), float(m.us_y)
    return p


class Oracle:
    """One FP64 lattice, initialised from a workload Case."""

    def __init__(self, case, threads: Optional[int] = None):
        L = lib()
        if threads:
            L.orc_set_threads(int(threads))
        self.case = case
        self.nx, self.ny = case.nx, case.ny
        self.params = make_params(case)
        self.h = L.orc_create(C.byref(self.params))
        if not self.h:
            raise ValueError("oracle: bad lattice size")
        for w in range(4):
            L.orc_set_wall_T(self.h, w, _ptr(case.wall_profile(w)))
        self._keep = [_f64(case.phi0), _f64(case.cos_theta), _f64(case.phi), _f64(case.T)]
        L.orc_init(self.h, *[_ptr(a) for a in self._keep])
        if getattr(case, "T_hold", None) is not None:
            self.set_isothermal(case.T_hold)

    def set_isothermal(self, T_hold) -> None:
        """Per-node held temperatures (NaN where free); None: the substrate rule."""
        if T_hold is None:
            lib().orc_set_isothermal(self.h, None)
            return
        self._thold = _f64(T_hold)
        lib().orc_set_isothermal(self.h, _ptr(self._thold))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def step(self, n: int = 1) -> None:
        lib().orc_step(self.h, int(n))

    def set_store_f32(self, on: bool) -> None:
        """Conditioning probe: round the state to binary32 after every step."""
        lib().orc_set_store_f32(self.h, int(bool(on)))

    def set_wall_T(self, wall: int, prof) -> None:
        lib().orc_set_wall_T(self.h, wall, _ptr(_f64(prof)))

    def set_cos_theta(self, cth) -> None:
        lib().orc_set_cos_theta(self.h, _ptr(_f64(cth)))

    def fields(self) -> Dict[str, np.ndarray]:
        n = self.nx * self.ny
        out = np.empty(len(FIELDS) * n)
        lib().orc_fields(self.h, _ptr(out))
        return {k: out[i * n:(i + 1) * n].reshape(self.ny, self.nx).copy()
                for i, k in enumerate(FIELDS)}

    def reduce(self) -> Dict[str, float]:
        out = np.empty(len(REDS))
        lib().orc_reduce(self.h, _ptr(out))
        return dict(zip(REDS, out.tolist()))

    def get_state(self):
        n = self.nx * self.ny
        f, g, h = (np.empty(9 * n) for _ in range(3))
        lag = np.empty(NLAG * n)
        lib().orc_get_state(self.h, _ptr(f), _ptr(g), _ptr(h), _ptr(lag))
        sh = (9, self.ny, self.nx)
        return f.reshape(sh), g.reshape(sh), h.reshape(sh), lag.reshape(NLAG, self.ny, self.nx)

    def set_state(self, f, g, h, lag) -> None:
        lib().orc_set_state(self.h, _ptr(_f64(f).ravel()), _ptr(_f64(g).ravel()),
                            _ptr(_f64(h).ravel()), _ptr(_f64(lag).ravel()))

    @property
    def step_count(self) -> int:
        return int(lib().orc_step_count(self.h))


# ---- per-node pieces for the algebra checks ---------------------------------

def feq(p, rho, ux, uy) -> np.ndarray:
    out = np.empty(9)
    lib().orc_feq(p, rho, ux, uy, _ptr(out))
    return out


def geq(phi, mu, jx, jy) -> np.ndarray:
    out = np.empty(9)
    lib().orc_geq(phi, mu, jx, jy, _ptr(out))
    return out


def heq(rhoH, T, rhocp, Eref, ux, uy) -> np.ndarray:
    out = np.empty(9)
    lib().orc_heq(rhoH, T, rhocp, Eref, ux, uy, _ptr(out))
    return out


def forcing(S, Fx, Fy, rfx, rfy, Ftx, Fty, ux, uy) -> np.ndarray:
    out = np.empty(9)
    lib().orc_forcing(S, Fx, Fy, rfx, rfy, Ftx, Fty, ux, uy, _ptr(out))
    return out


def hmap(case, rhoH, phi0, Cw, chi):
    out = np.empty(4)
    p = make_params(case)
    lib().orc_hmap(C.byref(p), rhoH, phi0, Cw, chi, _ptr(out))
    return dict(T=out[0], fl=out[1], Ksol=out[2], Kliq=out[3])


def chem_pot(case, phi, lap_phi, phi0, cth, lap_phi0, fs, lap_fs) -> float:
    """mu_phi of one node (the oracle's chemical potential)."""
    p = make_params(case)
    return float(lib().orc_chem_pot(C.byref(p), phi, lap_phi, phi0, cth, lap_phi0, fs, lap_fs))


def stencil(X: np.ndarray, periodic_x: bool, periodic_y: bool):
    X = _f64(X)
    ny, nx = X.shape
    gx, gy, lap = (np.empty_like(X) for _ in range(3))
    lib().orc_stencil(nx, ny, int(periodic_x), int(periodic_y), _ptr(X), _ptr(gx),
                      _ptr(gy), _ptr(lap))
    return gx, gy, lap
