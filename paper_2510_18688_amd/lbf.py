"""Python binding of liblbf (argument marshalling only).

Every step of the coupled update runs in the HIP kernels of liblbf.so; this
module converts arrays and tensors to pointers and sizes and raises on error
codes.  PyTorch provides device memory (the simulation workspace) and the
HIP stream.  There is no CPU fallback: without the built library, or
without a HIP device, every entry point raises.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbf.so")

FIELDS = ["phi", "T", "fl", "fs", "ux", "uy", "p", "rhoH", "mu", "C", "chi", "rho", "phihat"]
REDS = ["sum_g", "sum_h", "sum_fs", "sum_liq", "umax", "nonfinite", "src_phi", "src_heat",
        "wall_flux", "reset", "step"]
EXPORTS = ["lbf_workspace_bytes", "lbf_create", "lbf_set_geometry", "lbf_set_wall_temperature",
           "lbf_init_fields", "lbf_set_isothermal", "lbf_step", "lbf_read_field", "lbf_read_fields", "lbf_reduce",
           "lbf_set_poststream_state", "lbf_set_tile", "lbf_get_tile", "lbf_state_bytes", "lbf_save_state",
           "lbf_load_state", "lbf_set_timing", "lbf_last_step_kernel_ms", "lbf_copy_probe",
           "lbf_last_error",
           "lbf_destroy", "lbf_batch_create", "lbf_batch_set_tile", "lbf_batch_step",
           "lbf_batch_set_timing", "lbf_batch_last_step_ms", "lbf_batch_items",
           "lbf_batch_destroy", "lbf_tape_bytes", "lbf_tape_create", "lbf_tape_segment",
           "lbf_tape_forward", "lbf_tape_backward", "lbf_tape_destroy", "lbf_profiles",
           "lbf3_workspace_bytes", "lbf3_create", "lbf3_set_geometry", "lbf3_init_fields",
           "lbf3_step", "lbf3_read_fields", "lbf3_reduce", "lbf3_set_timing",
           "lbf3_last_step_ms", "lbf3_destroy", "lbf3_set_strip", "lbf3_state_bytes",
           "lbf3_save_state", "lbf3_load_state"]
COLS = ["ice", "pcm", "pcm_top", "ice_top"]
ROWS = ["ice", "pcm", "pcm_left", "pcm_right", "ice_left", "ice_right"]

ERRORS = {-1: "LBF_EINVAL", -2: "LBF_EHIP", -3: "LBF_ESTATE", -4: "LBF_EUNSTABLE",
          -5: "LBF_ENOMEM"}


class LbfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("periodic_x", C.c_int32),
                ("periodic_y", C.c_int32), ("thermal_bc", C.c_int32 * 4),
                ("latch_fs", C.c_int32), ("h_src_tau_a", C.c_int32),
                ("substrate_fixed", C.c_int32), ("plane_pad", C.c_int32)] + [
        (k, C.c_double) for k in (
            "rho_l", "rho_g", "rho_s", "mu_l", "mu_g", "mu_s", "lam_l", "lam_g", "lam_s",
            "cp_l", "cp_g", "cp_s", "latent", "T_m", "sigma", "eps", "mobility", "cos_psi",
            "rho_ref", "T_substrate", "pcm_floor")] + [
        ("mrt", C.c_int32), ("check_every", C.c_int32), ("phi_src_mdot", C.c_int32),
        ("row_block", C.c_int32), ("s_b", C.c_double), ("s_q", C.c_double),
        ("s_g", C.c_double), ("grav", C.c_double * 2), ("u_solid", C.c_double * 2)]


_lib = None


def load(path: str = LIB_PATH):
    """Load liblbf.so and declare its signatures (no GPU needed).

    torch is imported first so that the HIP runtime it carries is the one
    liblbf binds to (two runtimes in one process do not share devices)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"liblbf.so not built ({path}); run python -m paper_2510_18688_amd.build")
    L = C.CDLL(path)
    vp, i32, f_p, d_p = C.c_void_p, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_double)
    L.lbf_workspace_bytes.restype = C.c_size_t
    L.lbf_workspace_bytes.argtypes = [i32, i32, i32, i32]
    L.lbf_create.argtypes = [C.POINTER(Params), vp, vp, C.c_size_t, C.POINTER(vp)]
    L.lbf_set_geometry.argtypes = [vp, vp, vp, i32]
    L.lbf_set_wall_temperature.argtypes = [vp, i32, vp, i32, i32]
    L.lbf_set_isothermal.argtypes = [vp, vp, vp, i32]
    L.lbf_init_fields.argtypes = [vp, vp, vp, i32]
    L.lbf_set_poststream_state.argtypes = [vp, vp, vp, C.c_int64, i32]
    L.lbf_step.argtypes = [vp, i32]
    L.lbf_read_field.argtypes = [vp, i32, vp, i32]
    L.lbf_read_fields.argtypes = [vp, vp, i32]
    L.lbf_reduce.argtypes = [vp, d_p]
    L.lbf_set_tile.argtypes = [vp, i32, i32]
    L.lbf_get_tile.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    L.lbf_state_bytes.restype = C.c_size_t
    L.lbf_state_bytes.argtypes = [vp]
    L.lbf_save_state.argtypes = [vp, vp, C.c_size_t]
    L.lbf_load_state.argtypes = [vp, vp, C.c_size_t]
    L.lbf_set_timing.argtypes = [vp, i32]
    L.lbf_copy_probe.argtypes = [vp, i32, d_p, d_p]
    L.lbf_last_step_kernel_ms.restype = C.c_double
    L.lbf_last_step_kernel_ms.argtypes = [vp]
    L.lbf_last_error.restype = C.c_char_p
    L.lbf_destroy.argtypes = [vp]
    L.lbf_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(vp)]
    L.lbf_batch_set_tile.argtypes = [vp, i32, i32]
    L.lbf_batch_step.argtypes = [vp, i32]
    L.lbf_batch_set_timing.argtypes = [vp, i32]
    L.lbf_batch_last_step_ms.restype = C.c_double
    L.lbf_batch_last_step_ms.argtypes = [vp]
    L.lbf_batch_items.restype = i32
    L.lbf_batch_items.argtypes = [vp]
    L.lbf_batch_destroy.argtypes = [vp]
    L.lbf_tape_bytes.restype = C.c_size_t
    L.lbf_tape_bytes.argtypes = [i32, i32, i32, i32, i32]
    L.lbf_tape_create.argtypes = [vp, i32, i32, C.POINTER(vp)]
    L.lbf_tape_segment.restype = i32
    L.lbf_tape_segment.argtypes = [vp]
    L.lbf_tape_forward.argtypes = [vp]
    L.lbf_tape_backward.argtypes = [vp, vp, vp, vp, i32, vp, vp, i32]
    L.lbf_tape_destroy.argtypes = [vp]
    L.lbf_profiles.argtypes = [vp, vp, vp, i32]
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != 0:
        raise LbfError(rc, _lib.lbf_last_error().decode())


def make_params(case) -> Params:
    p = Params()
    p.nx, p.ny = case.nx, case.ny
    p.periodic_x, p.periodic_y = int(case.periodic_x), int(case.periodic_y)
    for w in range(4):
        p.thermal_bc[w] = int(case.thermal_bc[w])
    m = case.mat
    p.latch_fs, p.h_src_tau_a = int(m.latch_fs), int(m.h_src_tau_a)
    p.substrate_fixed = int(case.substrate_fixed)
    for k in ("rho_l", "rho_g", "rho_s", "mu_l", "mu_g", "mu_s", "lam_l", "lam_g", "lam_s",
              "cp_l", "cp_g", "cp_s", "latent", "T_m", "sigma", "eps", "mobility", "cos_psi",
              "rho_ref", "pcm_floor"):
        setattr(p, k, float(getattr(m, k)))
    p.T_substrate = float(case.T_substrate)
    p.mrt = int(getattr(m, "mrt", 0))
    p.phi_src_mdot = int(getattr(m, "phi_src_mdot", 0))
    p.s_b, p.s_q = float(getattr(m, "s_b", 0.0)), float(getattr(m, "s_q", 0.0))
    p.s_g = float(getattr(m, "s_g", 0.0))
    p.grav[0], p.grav[1] = float(m.g_x), float(m.g_y)
    p.u_solid[0], p.u_solid[1] = float(m.us_x), float(m.us_y)
    return p


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("liblbf needs a HIP device; none is visible")
    return torch


def _f32_host(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


class Sim:
    """One lattice on the current HIP device; workspace owned by a torch tensor.

    `tile` is the launch shape (threads along x, rows per block),
    `row_block` the state's memory layout (0 plane-major; 1 .. 32 rows per
    block of all planes, lbf_params.row_block) and `plane_pad` the padding
    between its planes in floats (a multiple of 64); they change speed only,
    and `autotune.lookup` / `autotune.lookup_layout` return the tuned values
    for a lattice size (row_block None takes the latter's).  The adjoint
    (`Tape`) needs row_block 0.
    `check_every`: `step` raises LbfError(LBF_EUNSTABLE) after a step that
    starts at a time level divisible by it found a non-finite or too fast
    state (0: no checks)."""

    def __init__(self, case, tile: Optional[Sequence[int]] = None, device: str = "cuda",
                 stream=None, plane_pad: int = 0, check_every: int = 1000,
                 row_block: Optional[int] = None):
        torch = _torch()
        L = load()
        self.case = case
        self.nx, self.ny = case.nx, case.ny
        self.params = make_params(case)
        self.params.plane_pad = int(plane_pad)
        if row_block is None:
            from . import autotune
            row_block = autotune.lookup_layout(self.nx, self.ny)[0]
        self.params.row_block = int(row_block)
        self.params.check_every = int(check_every)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = L.lbf_workspace_bytes(self.nx, self.ny, self.params.plane_pad,
                                       self.params.row_block)
        if nbytes == 0:
            raise LbfError(-1, f"bad lattice size {self.nx} x {self.ny}, plane_pad {plane_pad} "
                               f"or row_block {row_block}")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        check(L.lbf_create(C.byref(self.params), C.c_void_p(self.stream.cuda_stream),
                           C.c_void_p(self.workspace.data_ptr()), nbytes, C.byref(h)))
        self.h = h
        if tile is not None:
            self.set_tile(*tile)
        self.set_geometry(case.phi0, case.cos_theta)
        for w in range(4):
            self.set_wall_temperature(w, case.wall_profile(w))
        if getattr(case, "T_hold", None) is not None:
            self.set_isothermal(np.isfinite(case.T_hold), np.nan_to_num(case.T_hold))
        self.init_fields(case.phi, case.T)

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.lbf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- marshalling helpers
    def _ptr_in(self, a):
        """(pointer, on_device, keep-alive) for a host array or a device tensor."""
        try:
            import torch
            if isinstance(a, torch.Tensor):
                if a.device.type != "cuda" or a.dtype != torch.float32 or not a.is_contiguous():
                    raise LbfError(-1, "tensor inputs must be contiguous float32 on the device")
                return C.c_void_p(a.data_ptr()), 1, a
        except ImportError:
            pass
        arr = _f32_host(a)
        return C.c_void_p(arr.ctypes.data), 0, arr

    def set_geometry(self, phi0, cos_theta) -> None:
        a, d, k1 = self._ptr_in(phi0)
        b, d2, k2 = self._ptr_in(cos_theta)
        if d != d2:
            raise LbfError(-1, "phi0 and cos_theta must both be host or both device")
        check(_lib.lbf_set_geometry(self.h, a, b, d))

    def set_isothermal(self, mask, T_hold) -> None:
        """Hold the nodes where `mask` is true at the temperatures `T_hold`
        ([ny, nx] host arrays or device tensors: uint8/bool mask, float32
        temperatures); mask None removes the per-node region."""
        if mask is None:
            check(_lib.lbf_set_isothermal(self.h, None, None, 0))
            return
        import torch
        if isinstance(mask, torch.Tensor):
            if mask.device.type != "cuda" or mask.dtype not in (torch.uint8, torch.bool) \
                    or not mask.is_contiguous() or mask.numel() != self.nx * self.ny:
                raise LbfError(-1, "mask tensor: contiguous uint8/bool, nx * ny, on the device")
            m, dm = C.c_void_p(mask.data_ptr()), 1
            keep = mask
        else:
            keep = np.ascontiguousarray(np.asarray(mask).reshape(-1) != 0, dtype=np.uint8)
            if keep.size != self.nx * self.ny:
                raise LbfError(-1, "mask needs nx * ny values")
            m, dm = C.c_void_p(keep.ctypes.data), 0
        t, dt, k2 = self._ptr_in(T_hold)
        if dm != dt:
            raise LbfError(-1, "mask and T_hold must both be host or both device")
        check(_lib.lbf_set_isothermal(self.h, m, t, dm))
        del keep, k2

    def set_wall_temperature(self, wall: int, Tw) -> None:
        a, d, k = self._ptr_in(Tw)
        n = self.nx if wall in (0, 1) else self.ny
        check(_lib.lbf_set_wall_temperature(self.h, wall, a, n, d))

    def init_fields(self, phi, T) -> None:
        a, d, k1 = self._ptr_in(phi)
        b, d2, k2 = self._ptr_in(T)
        if d != d2:
            raise LbfError(-1, "phi and T must both be host or both device")
        check(_lib.lbf_init_fields(self.h, a, b, d))

    def set_poststream_state(self, f, g, h, lag, step: int = 0) -> None:
        """Load post-streaming distributions (9 planes each) and lagged fields
        (7: f_s, Q, (phi u)_x, (phi u)_y, p, u_x, u_y)."""
        dist = np.ascontiguousarray(np.concatenate([np.reshape(f, (9, -1)), np.reshape(g, (9, -1)),
                                                    np.reshape(h, (9, -1))]), dtype=np.float32)
        lg = np.ascontiguousarray(np.reshape(lag, (7, -1)), dtype=np.float32)
        check(_lib.lbf_set_poststream_state(self.h, C.c_void_p(dist.ctypes.data),
                                            C.c_void_p(lg.ctypes.data), int(step), 0))

    def set_tile(self, tx: int, ty: int) -> None:
        check(_lib.lbf_set_tile(self.h, int(tx), int(ty)))

    def tile(self):
        a, b = C.c_int32(), C.c_int32()
        check(_lib.lbf_get_tile(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def step(self, n: int = 1) -> None:
        check(_lib.lbf_step(self.h, int(n)))

    def set_timing(self, on: bool) -> None:
        check(_lib.lbf_set_timing(self.h, int(bool(on))))

    def copy_probe(self, launches: int = 20):
        """(ms per launch, bytes per launch) of a copy of the planes a step
        reads and writes, in the step kernel's own tile and row order: the
        bandwidth ceiling of its access pattern (the state is unchanged)."""
        ms, nb = C.c_double(), C.c_double()
        check(_lib.lbf_copy_probe(self.h, int(launches), C.byref(ms), C.byref(nb)))
        return ms.value, nb.value

    def last_step_kernel_ms(self) -> float:
        return float(_lib.lbf_last_step_kernel_ms(self.h))

    def fields(self) -> Dict[str, np.ndarray]:
        n = self.nx * self.ny
        out = np.empty(len(FIELDS) * n, dtype=np.float32)
        check(_lib.lbf_read_fields(self.h, C.c_void_p(out.ctypes.data), 0))
        return {k: out[i * n:(i + 1) * n].reshape(self.ny, self.nx) for i, k in enumerate(FIELDS)}

    def field(self, name: str, out=None):
        """One read-out field into a new host array, or into a device tensor `out`."""
        fid = FIELDS.index(name)
        if out is not None:
            check(_lib.lbf_read_field(self.h, fid, C.c_void_p(out.data_ptr()), 1))
            return out
        arr = np.empty((self.ny, self.nx), dtype=np.float32)
        check(_lib.lbf_read_field(self.h, fid, C.c_void_p(arr.ctypes.data), 0))
        return arr

    def reduce(self, check_stable: bool = True) -> Dict[str, float]:
        out = (C.c_double * len(REDS))()
        rc = _lib.lbf_reduce(self.h, out)
        if rc != 0 and (check_stable or rc != -4):
            check(rc)
        return dict(zip(REDS, list(out)))

    def profiles(self) -> Dict[str, Dict[str, np.ndarray]]:
        """Column and row profiles of the current state (FP64): {"col": {ice,
        pcm, pcm_top, ice_top} each [nx], "row": {ice, pcm, pcm_left,
        pcm_right, ice_left, ice_right} each [ny]}."""
        col = np.empty(len(COLS) * self.nx)
        row = np.empty(len(ROWS) * self.ny)
        check(_lib.lbf_profiles(self.h, C.c_void_p(col.ctypes.data), C.c_void_p(row.ctypes.data), 0))
        return {"col": {k: col[i * self.nx:(i + 1) * self.nx] for i, k in enumerate(COLS)},
                "row": {k: row[i * self.ny:(i + 1) * self.ny] for i, k in enumerate(ROWS)}}

    def state_bytes(self) -> int:
        return int(_lib.lbf_state_bytes(self.h))

    def _state_buffer(self, buf):
        """Pointer and size of a checkpoint buffer: contiguous device memory of
        at least state_bytes() bytes (the library copies device to device)."""
        import torch
        if not isinstance(buf, torch.Tensor) or buf.device.type != "cuda" or not buf.is_contiguous():
            raise LbfError(-1, "a state buffer must be a contiguous tensor in device memory")
        nbytes = buf.numel() * buf.element_size()
        if nbytes < self.state_bytes():
            raise LbfError(-5, f"state buffer of {nbytes} bytes, {self.state_bytes()} needed")
        return C.c_void_p(buf.data_ptr()), nbytes

    def save_state(self, buf) -> None:
        ptr, nbytes = self._state_buffer(buf)
        check(_lib.lbf_save_state(self.h, ptr, nbytes))

    def load_state(self, buf) -> None:
        ptr, nbytes = self._state_buffer(buf)
        check(_lib.lbf_load_state(self.h, ptr, nbytes))


class Batch:
    """Many lattices advanced together by one persistent launch per step."""

    def __init__(self, sims: Sequence[Sim], tile: Optional[Sequence[int]] = None):
        L = load()
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s.h.value for s in self.sims])
        h = C.c_void_p()
        check(L.lbf_batch_create(arr, len(self.sims), C.byref(h)))
        self.h = h
        if tile is not None:
            self.set_tile(*tile)

    def set_tile(self, tx: int, ty: int) -> None:
        check(_lib.lbf_batch_set_tile(self.h, int(tx), int(ty)))

    def step(self, n: int = 1) -> None:
        check(_lib.lbf_batch_step(self.h, int(n)))

    def set_timing(self, on: bool) -> None:
        check(_lib.lbf_batch_set_timing(self.h, int(bool(on))))

    def last_step_ms(self) -> float:
        return float(_lib.lbf_batch_last_step_ms(self.h))

    def items(self) -> int:
        return int(_lib.lbf_batch_items(self.h))

    @property
    def nodes(self) -> int:
        return sum(s.nx * s.ny for s in self.sims)

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.lbf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tape:
    """Reverse-mode differentiation of a run of `nsteps` steps of `sim` with a
    checkpoint every `segment` steps (0: ceil(sqrt(nsteps)))."""

    def __init__(self, sim: Sim, nsteps: int, segment: int = 0):
        L = load()
        self.sim = sim
        self.nsteps = int(nsteps)
        h = C.c_void_p()
        check(L.lbf_tape_create(sim.h, self.nsteps, int(segment), C.byref(h)))
        self.h = h

    @property
    def segment(self) -> int:
        return int(_lib.lbf_tape_segment(self.h))

    def forward(self) -> None:
        check(_lib.lbf_tape_forward(self.h))

    def backward(self, seed_phi=None, seed_T=None, seed_fs=None):
        """Seeds dJ/dphi, dJ/dT, dJ/df_s of the final state ([ny, nx]; device
        float32 tensors or host arrays, None = 0).  Returns the FP64 device
        tensors dJ/dcos(theta) [ny, nx] and dJ/dT_w [2 nx + 2 ny] (bottom, top,
        left, right)."""
        import torch
        seeds = [seed_phi, seed_T, seed_fs]
        dev = [isinstance(a, torch.Tensor) for a in seeds if a is not None]
        if dev and not (all(dev) or not any(dev)):
            raise LbfError(-1, "seeds must all be device tensors or all host arrays")
        on_dev = int(bool(dev) and dev[0])
        ptrs, keep = [], []
        for a in seeds:
            if a is None:
                ptrs.append(None)
                continue
            if on_dev:
                if a.device.type != "cuda" or a.dtype != torch.float32 or not a.is_contiguous():
                    raise LbfError(-1, "seed tensors must be contiguous float32 on the device")
                if a.numel() != self.sim.nx * self.sim.ny:
                    raise LbfError(-1, "a seed needs nx * ny values")
                ptrs.append(C.c_void_p(a.data_ptr()))
                keep.append(a)
            else:
                arr = _f32_host(a).reshape(-1)
                if arr.size != self.sim.nx * self.sim.ny:
                    raise LbfError(-1, "a seed needs nx * ny values")
                ptrs.append(C.c_void_p(arr.ctypes.data))
                keep.append(arr)
        nx, ny = self.sim.nx, self.sim.ny
        gc = torch.empty((ny, nx), dtype=torch.float64, device=self.sim.device)
        gw = torch.empty(2 * nx + 2 * ny, dtype=torch.float64, device=self.sim.device)
        check(_lib.lbf_tape_backward(self.h, ptrs[0], ptrs[1], ptrs[2], on_dev,
                                     C.c_void_p(gc.data_ptr()), C.c_void_p(gw.data_ptr()), 1))
        return gc, gw

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.lbf_tape_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wall_vector(case):
    """The wall temperatures of a case as one vector [2 nx + 2 ny]: bottom,
    top, left, right."""
    return np.concatenate([np.broadcast_to(np.asarray(case.wall_profile(w), dtype=np.float64),
                                           (case.nx if w < 2 else case.ny,))
                           for w in range(4)])


def _freeze_function():
    import torch

    class FreezeFields(torch.autograd.Function):
        """(cos theta per node [ny, nx], wall temperatures [2 nx + 2 ny]) ->
        (phi, T, f_s) [ny, nx] after `steps` coupled steps from the case's
        initial fields.  The backward pass is the library's adjoint sweep."""

        @staticmethod
        def forward(ctx, cos_theta, wall_T, case, steps, segment, tile):
            sim = Sim(case, tile=tile, row_block=0)
            dev = sim.device
            sim.set_geometry(torch.as_tensor(np.ascontiguousarray(case.phi0, dtype=np.float32),
                                             device=dev),
                             cos_theta.detach().to(device=dev, dtype=torch.float32).contiguous())
            wt = wall_T.detach().to(device=dev, dtype=torch.float32).contiguous()
            nx, ny = case.nx, case.ny
            bounds = [0, nx, 2 * nx, 2 * nx + ny, 2 * nx + 2 * ny]
            for w in range(4):
                sim.set_wall_temperature(w, wt[bounds[w]:bounds[w + 1]].contiguous())
            sim.init_fields(torch.as_tensor(np.ascontiguousarray(case.phi, dtype=np.float32),
                                            device=dev),
                            torch.as_tensor(np.ascontiguousarray(case.T, dtype=np.float32),
                                            device=dev))
            tape = Tape(sim, steps, segment)
            tape.forward()
            out = [sim.field(k, torch.empty((ny, nx), dtype=torch.float32, device=dev))
                   for k in ("phi", "T", "fs")]
            ctx.tape = tape
            ctx.dtypes = (cos_theta.dtype, wall_T.dtype, cos_theta.device, wall_T.device)
            return tuple(out)

        @staticmethod
        def backward(ctx, g_phi, g_T, g_fs):
            def seed(g):
                return None if g is None else g.detach().to(torch.float32).contiguous()
            gc, gw = ctx.tape.backward(seed(g_phi), seed(g_T), seed(g_fs))
            ctx.tape.close()
            ct, wt, cd, wd = ctx.dtypes
            return gc.to(device=cd, dtype=ct), gw.to(device=wd, dtype=wt), None, None, None, None

    return FreezeFields


_FREEZE = None


def freeze_fields(cos_theta, wall_T, case, steps: int, segment: int = 0, tile=None):
    """Differentiable run: see FreezeFields."""
    global _FREEZE
    if _FREEZE is None:
        _FREEZE = _freeze_function()
    return _FREEZE.apply(cos_theta, wall_T, case, int(steps), int(segment), tile)


# ---------------------------------------------------------------- 3D (D3Q19)
FIELDS3 = ["phi", "T", "fl", "fs", "ux", "uy", "uz", "p", "rhoH", "mu", "C", "chi", "rho",
           "phihat"]


class Params3(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_int32 * 3), ("thermal_bc", C.c_int32 * 6),
                ("latch_fs", C.c_int32), ("h_src_tau_a", C.c_int32),
                ("substrate_fixed", C.c_int32), ("plane_pad", C.c_int32)] + [
        (k, C.c_double) for k in (
            "rho_l", "rho_g", "rho_s", "mu_l", "mu_g", "mu_s", "lam_l", "lam_g", "lam_s",
            "cp_l", "cp_g", "cp_s", "latent", "T_m", "sigma", "eps", "mobility", "cos_psi",
            "rho_ref", "T_substrate", "pcm_floor")] + [
        ("wall_T", C.c_double * 6), ("grav", C.c_double * 3), ("u_solid", C.c_double * 3),
        ("phi_src_mdot", C.c_int32), ("row_block", C.c_int32)]


def _declare3(L):
    if getattr(L, "_lbf3_declared", False):
        return
    vp, i32 = C.c_void_p, C.c_int32
    L.lbf3_workspace_bytes.restype = C.c_size_t
    L.lbf3_workspace_bytes.argtypes = [i32, i32, i32, i32, i32]
    L.lbf3_create.argtypes = [C.POINTER(Params3), vp, vp, C.c_size_t, C.POINTER(vp)]
    L.lbf3_set_geometry.argtypes = [vp, vp, vp, i32]
    L.lbf3_init_fields.argtypes = [vp, vp, vp, i32]
    L.lbf3_step.argtypes = [vp, i32]
    L.lbf3_read_fields.argtypes = [vp, vp, i32]
    L.lbf3_reduce.argtypes = [vp, C.POINTER(C.c_double)]
    L.lbf3_set_timing.argtypes = [vp, i32]
    L.lbf3_set_strip.argtypes = [vp, i32]
    L.lbf3_state_bytes.restype = C.c_size_t
    L.lbf3_state_bytes.argtypes = [vp]
    L.lbf3_save_state.argtypes = [vp, vp, C.c_size_t]
    L.lbf3_load_state.argtypes = [vp, vp, C.c_size_t]
    L.lbf3_last_step_ms.restype = C.c_double
    L.lbf3_last_step_ms.argtypes = [vp]
    L.lbf3_destroy.argtypes = [vp]
    L._lbf3_declared = True


def make_params3(case) -> Params3:
    p = Params3()
    p.nx, p.ny, p.nz = case.nx, case.ny, case.nz
    for a in range(3):
        p.periodic[a] = int(bool(case.periodic[a]))
    for f in range(6):
        p.thermal_bc[f] = int(case.thermal_bc[f])
        p.wall_T[f] = float(case.wall_T[f])
    m = case.mat
    p.latch_fs, p.h_src_tau_a = int(m.latch_fs), int(m.h_src_tau_a)
    p.substrate_fixed = int(case.substrate_fixed)
    for k in ("rho_l", "rho_g", "rho_s", "mu_l", "mu_g", "mu_s", "lam_l", "lam_g", "lam_s",
              "cp_l", "cp_g", "cp_s", "latent", "T_m", "sigma", "eps", "mobility", "cos_psi",
              "rho_ref", "pcm_floor"):
        setattr(p, k, float(getattr(m, k)))
    p.T_substrate = float(case.T_substrate)
    for a, k in enumerate("xyz"):
        p.grav[a] = float(getattr(m, "g_" + k))
        p.u_solid[a] = float(getattr(m, "us_" + k))
    p.phi_src_mdot = int(getattr(m, "phi_src_mdot", 0))
    return p


class Sim3:
    """One D3Q19 lattice on the current HIP device (workspace: a torch tensor);
    `row_block` the state's memory layout (0 plane-major; 1 .. 64 rows of nx
    nodes per block of all planes, lbf3_params.row_block) and `plane_pad` its
    padding, as for `Sim` (`autotune.lookup_layout3(nx, ny, nz)`)."""

    def __init__(self, case, device: str = "cuda", stream=None, plane_pad: int = 0,
                 row_block: int = 32):
        torch = _torch()
        L = load()
        _declare3(L)
        self.case = case
        self.shape = (case.nz, case.ny, case.nx)
        self.params = make_params3(case)
        self.params.plane_pad = int(plane_pad)
        self.params.row_block = int(row_block)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = L.lbf3_workspace_bytes(case.nx, case.ny, case.nz, self.params.plane_pad,
                                        self.params.row_block)
        if nbytes == 0:
            raise LbfError(-1, f"bad lattice size {self.shape}, plane_pad {plane_pad} or "
                               f"row_block {row_block}")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        check(L.lbf3_create(C.byref(self.params), C.c_void_p(self.stream.cuda_stream),
                            C.c_void_p(self.workspace.data_ptr()), nbytes, C.byref(h)))
        self.h = h
        a, b = _f32_host(case.phi0), _f32_host(case.cos_theta)
        check(L.lbf3_set_geometry(self.h, C.c_void_p(a.ctypes.data), C.c_void_p(b.ctypes.data), 0))
        a, b = _f32_host(case.phi), _f32_host(case.T)
        check(L.lbf3_init_fields(self.h, C.c_void_p(a.ctypes.data), C.c_void_p(b.ctypes.data), 0))

    def step(self, n: int = 1) -> None:
        check(_lib.lbf3_step(self.h, int(n)))

    def state_bytes(self) -> int:
        return int(_lib.lbf3_state_bytes(self.h))

    def save_state(self, buf) -> None:
        ptr, nbytes = Sim._state_buffer(self, buf)
        check(_lib.lbf3_save_state(self.h, ptr, nbytes))

    def load_state(self, buf) -> None:
        ptr, nbytes = Sim._state_buffer(self, buf)
        check(_lib.lbf3_load_state(self.h, ptr, nbytes))

    def set_strip(self, rows: int) -> None:
        """Rows per strip of the step kernel's node order (>= ny: x-fastest)."""
        check(_lib.lbf3_set_strip(self.h, int(rows)))

    def set_timing(self, on: bool) -> None:
        check(_lib.lbf3_set_timing(self.h, int(bool(on))))

    def last_step_ms(self) -> float:
        return float(_lib.lbf3_last_step_ms(self.h))

    def fields(self) -> Dict[str, np.ndarray]:
        n = int(np.prod(self.shape))
        out = np.empty(len(FIELDS3) * n, dtype=np.float32)
        check(_lib.lbf3_read_fields(self.h, C.c_void_p(out.ctypes.data), 0))
        return {k: out[i * n:(i + 1) * n].reshape(self.shape) for i, k in enumerate(FIELDS3)}

    def reduce(self, check_stable: bool = True) -> Dict[str, float]:
        out = (C.c_double * len(REDS))()
        rc = _lib.lbf3_reduce(self.h, out)
        if rc != 0 and (check_stable or rc != -4):
            check(rc)
        return dict(zip(REDS, list(out)))

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.lbf3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
