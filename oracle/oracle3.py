"""ctypes front end of the FP64 D3Q19 oracle (test infrastructure only).

lbf_oracle3.c is the coupled step of Sec. 3 on the nineteen-velocity
lattice; this module builds it, marshals arrays and names the outputs.  Only
tests, the smoke check and the benchmark's CPU baseline may use it.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbf_oracle3.c")
LIB = os.path.join(HERE, "liblbf_oracle3.so")

FIELDS = ["phi", "T", "fl", "fs", "ux", "uy", "uz", "p", "rhoH", "mu", "C", "chi", "rho",
          "phihat"]
REDS = ["sum_g", "sum_h", "sum_fs", "sum_liq", "umax", "nonfinite",
        "src_phi", "src_heat", "wall_flux", "reset", "step"]


class Orc3Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_int32 * 3), ("thermal_bc", C.c_int32 * 6),
                ("latch_fs", C.c_int32), ("h_src_tau_a", C.c_int32),
                ("substrate_fixed", C.c_int32), ("pad_", C.c_int32)] + [
        (k, C.c_double) for k in (
            "rho_l", "rho_g", "rho_s", "mu_l", "mu_g", "mu_s", "lam_l", "lam_g", "lam_s",
            "cp_l", "cp_g", "cp_s", "latent", "T_m", "sigma", "eps", "mobility",
            "cos_psi", "rho_ref", "T_substrate", "pcm_floor")] + [
        ("wall_T", C.c_double * 6), ("grav", C.c_double * 3), ("u_solid", C.c_double * 3),
        ("phi_src_mdot", C.c_int32), ("pad2_", C.c_int32)]


def build(force: bool = False) -> str:
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
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.orc3_create.restype = C.c_void_p
        L.orc3_create.argtypes = [C.POINTER(Orc3Params)]
        L.orc3_destroy.argtypes = [C.c_void_p]
        L.orc3_init.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc3_step.argtypes = [C.c_void_p, C.c_int]
        L.orc3_fields.argtypes = [C.c_void_p, dp]
        L.orc3_reduce.argtypes = [C.c_void_p, dp]
        L.orc3_feq.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc3_geq.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc3_heq.argtypes = [C.c_double] * 4 + [dp, dp]
        L.orc3_forcing.argtypes = [C.c_double, dp, dp, dp, dp, dp]
        L.orc3_lattice.argtypes = [ip, dp, ip]
        L.orc3_stencil.argtypes = [C.c_int] * 3 + [ip, dp, dp, dp, dp, dp]
        L.orc3_set_threads.argtypes = [C.c_int]
        L.orc3_step_count.restype = C.c_long
        L.orc3_step_count.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(case) -> Orc3Params:
    p = Orc3Params()
    p.nx, p.ny, p.nz = case.nx, case.ny, case.nz
    for a in range(3):
        p.periodic[a] = int(bool(case.periodic[a]))
    for f in range(6):
        p.thermal_bc[f] = int(case.thermal_bc[f])
        p.wall_T[f] = float(case.wall_T[f])
    m = case.mat
    p.latch_fs, p.h_src_tau_a = int(m.latch_fs), int(m.h_src_tau_a)
    p.substrate_fixed = int(case.substrate_fixed)
    for k in ("rho_l", "rho_g", "rho_s", "mu_l", "mu_g", "mu_s", "lam_l", "lam_g",
              "lam_s", "cp_l", "cp_g", "cp_s", "latent", "T_m", "sigma", "eps",
              "mobility", "cos_psi", "rho_ref", "pcm_floor"):
        setattr(p, k, float(getattr(m, k)))
    p.T_substrate = float(case.T_substrate)
    for a, k in enumerate("xyz"):
        p.grav[a] = float(getattr(m, "g_" + k))
        p.u_solid[a] = float(getattr(m, "us_" + k))
    p.phi_src_mdot = int(getattr(m, "phi_src_mdot", 0))
    return p


class Oracle3:
    """One FP64 D3Q19 lattice, initialised from a Case3."""

    def __init__(self, case, threads: Optional[int] = None):
        L = lib()
        if threads:
            L.orc3_set_threads(int(threads))
        self.case = case
        self.shape = (case.nz, case.ny, case.nx)
        self.params = make_params(case)
        self.h = L.orc3_create(C.byref(self.params))
        if not self.h:
            raise ValueError("oracle: bad lattice size")
        self._keep = [_f64(case.phi0), _f64(case.cos_theta), _f64(case.phi), _f64(case.T)]
        L.orc3_init(self.h, *[_ptr(a) for a in self._keep])

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc3_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def step(self, n: int = 1) -> None:
        lib().orc3_step(self.h, int(n))

    @property
    def step_count(self) -> int:
        return int(lib().orc3_step_count(self.h))

    def fields(self) -> Dict[str, np.ndarray]:
        n = int(np.prod(self.shape))
        out = np.empty(len(FIELDS) * n)
        lib().orc3_fields(self.h, _ptr(out))
        return {k: out[i * n:(i + 1) * n].reshape(self.shape) for i, k in enumerate(FIELDS)}

    def reduce(self) -> Dict[str, float]:
        out = np.empty(len(REDS))
        lib().orc3_reduce(self.h, _ptr(out))
        return dict(zip(REDS, out.tolist()))
