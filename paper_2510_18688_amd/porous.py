"""Porous pre-processing on the GPU (binding of include/lbf_pre.h).

Sec. 4.6 prepares an unsaturated porous medium in two stages before
freezing it: the binary grain image is smoothed into the diffuse solid
indicator phi0 by a finite-time Cahn-Hilliard evolution (`ch_smooth`, the
liblbf kernels), and the liquid is distributed by spontaneous phase
separation of the uniform pore mixture phi = (1 - phi0) phi_i above the
melting point (the coupled step itself, `Sim.step`).  `prepare` runs both and
returns the simulation, ready for the freezing stage.
"""

from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import lbf


class ChParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_int32 * 3), ("A", C.c_double), ("kappa", C.c_double),
                ("mobility", C.c_double), ("dt", C.c_double)]


EXPORTS = ["lbf_ch_workspace_bytes", "lbf_ch_smooth", "lbf_ch_noalloc_max_nodes",
           "lbf_ch_smooth_noalloc"]


def _declare(L):
    if getattr(L, "_ch_declared", False):
        return
    i32, vp = C.c_int32, C.c_void_p
    L.lbf_ch_workspace_bytes.restype = C.c_size_t
    L.lbf_ch_workspace_bytes.argtypes = [i32, i32, i32]
    L.lbf_ch_smooth.argtypes = [C.POINTER(ChParams), vp, i32, vp, i32, i32, vp, vp, C.c_size_t]
    L.lbf_ch_noalloc_max_nodes.restype = C.c_size_t
    L.lbf_ch_noalloc_max_nodes.argtypes = []
    L.lbf_ch_smooth_noalloc.argtypes = [C.POINTER(ChParams), vp, vp, i32, vp]
    L._ch_declared = True


def ch_params(shape: Sequence[int], periodic: Sequence[bool], eps: float = 4.0, A: float = 1.0,
              mobility: float = 1.0, dt: float = 0.02) -> ChParams:
    """Parameters for an image of shape (ny, nx) or (nz, ny, nx); kappa =
    A eps^2 / 8 gives the flat equilibrium tanh(2 d / eps)."""
    shape = tuple(int(v) for v in shape)
    p = ChParams()
    if len(shape) == 2:
        p.nx, p.ny, p.nz = shape[1], shape[0], 1
    else:
        p.nx, p.ny, p.nz = shape[2], shape[1], shape[0]
    for a in range(3):
        p.periodic[a] = int(bool(periodic[a])) if a < len(periodic) else 1
    p.A, p.kappa, p.mobility, p.dt = A, A * eps * eps / 8.0, mobility, dt
    return p


def ch_smooth(solid, periodic: Sequence[bool], iterations: int, eps: float = 4.0,
              A: float = 1.0, mobility: float = 1.0, dt: float = 0.02, stream=None,
              workspace=None):
    """phi0 (float32) of a binary image after `iterations` Euler steps of the
    Cahn-Hilliard equation on the GPU.  `solid`: numpy array (host; the
    result is numpy) or a uint8 torch tensor on the device (the result is a
    float32 tensor on the same device)."""
    torch = lbf._torch()
    L = lbf.load()
    _declare(L)
    on_dev = hasattr(solid, "data_ptr")
    shape = tuple(solid.shape)
    p = ch_params(shape, periodic, eps, A, mobility, dt)
    need = L.lbf_ch_workspace_bytes(p.nx, p.ny, p.nz)
    if need == 0:
        raise lbf.LbfError(-1, f"bad image shape {shape}")
    if stream is None:
        stream = torch.cuda.current_stream()
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    if on_dev:
        if solid.dtype != torch.uint8 or not solid.is_contiguous():
            raise ValueError("a device image must be a contiguous uint8 tensor")
        out = torch.empty(shape, dtype=torch.float32, device=solid.device)
        src, dst = C.c_void_p(solid.data_ptr()), C.c_void_p(out.data_ptr())
    else:
        host = np.ascontiguousarray(np.asarray(solid) != 0, dtype=np.uint8)
        out = np.empty(shape, dtype=np.float32)
        src, dst = C.c_void_p(host.ctypes.data), C.c_void_p(out.ctypes.data)
    lbf.check(L.lbf_ch_smooth(C.byref(p), src, int(on_dev), dst, int(on_dev), int(iterations),
                              C.c_void_p(stream.cuda_stream), C.c_void_p(workspace.data_ptr()),
                              workspace.numel()))
    return out


def ch_smooth_noalloc(solid, out, periodic: Sequence[bool], iterations: int, eps: float = 4.0,
                      A: float = 1.0, mobility: float = 1.0, dt: float = 0.02, stream=None):
    """`ch_smooth` through the allocation-free entry point: `solid` is a
    contiguous uint8 device tensor, `out` a contiguous float32 device tensor
    of the same shape that receives phi0; the library's per-device scratch
    holds the working planes (images of up to lbf_ch_noalloc_max_nodes()
    nodes).  Ordered on `stream` (default: torch's current stream); returns
    `out`."""
    torch = lbf._torch()
    L = lbf.load()
    _declare(L)
    if not (hasattr(solid, "data_ptr") and hasattr(out, "data_ptr")):
        raise ValueError("solid and out must be device tensors")
    if solid.dtype != torch.uint8 or not solid.is_contiguous() or solid.device.type != "cuda":
        raise ValueError("solid must be a contiguous uint8 device tensor")
    if out.dtype != torch.float32 or not out.is_contiguous() or out.shape != solid.shape \
            or out.device != solid.device:
        raise ValueError("out must be a contiguous float32 tensor of the image's shape and device")
    p = ch_params(tuple(solid.shape), periodic, eps, A, mobility, dt)
    if stream is None:
        stream = torch.cuda.current_stream(solid.device)
    with torch.cuda.device(solid.device):
        lbf.check(L.lbf_ch_smooth_noalloc(C.byref(p), C.c_void_p(solid.data_ptr()),
                                          C.c_void_p(out.data_ptr()), int(iterations),
                                          C.c_void_p(stream.cuda_stream)))
    return out


def prepare(solid: np.ndarray, S_w: float, theta_deg: float, ch_iterations: int = 500,
            separation_steps: int = 2000, eps: Optional[float] = None, T0: float = 0.5,
            tile=None, gravity=(0.0, 0.0)):
    """Both pre-processing stages of Sec. 4.6 on a 2D image (ny, nx), walls
    on all sides: smooth it into phi0, fill the pores with the uniform
    mixture of saturation S_w, and let it separate for `separation_steps`
    steps at T0 (above melting) under the body force rho * gravity.  Returns
    (sim, case); set the freezing stage's wall temperatures with
    `sim.set_wall_temperature` and step on."""
    from . import workloads as W
    mat = W.Material()
    phi0 = ch_smooth(solid, (False, False, True), ch_iterations, eps=eps or mat.eps)
    case = W.unsaturated_medium(phi0.astype(np.float64), S_w=S_w, theta_deg=theta_deg, T0=T0,
                                mat=mat, gravity=gravity)
    sim = lbf.Sim(case, tile=tile)
    sim.step(separation_steps)
    return sim, case
