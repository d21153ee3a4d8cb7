"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point that include/lbf.h, include/lbf3.h and include/lbf_pre.h
declare, the parameter structs match the binding's, and parameter validation rejects bad sets
before touching a device."""

import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_2510_18688_amd import lbf, workloads as W, workloads3 as W3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("lbf.h", "lbf3.h", "lbf_pre.h")]


@pytest.fixture(scope="module")
def L():
    from paper_2510_18688_amd import build
    if build.stale():
        build.build(verbose=False)
    return lbf.load()


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(lbf3?_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 27 and "lbf3_step" in names and "lbf_ch_smooth" in names
    for n in names:
        assert hasattr(L, n), n
    from paper_2510_18688_amd import porous
    assert set(lbf.EXPORTS) | set(porous.EXPORTS) == set(names)


def test_params_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbf.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lbf_params),'
                   ' offsetof(lbf_params, rho_l), offsetof(lbf_params, T_substrate),'
                   ' offsetof(lbf_params, thermal_bc), offsetof(lbf_params, mrt),'
                   ' offsetof(lbf_params, s_q), offsetof(lbf_params, check_every),'
                   ' offsetof(lbf_params, phi_src_mdot));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    P = lbf.Params
    assert int(out[0]) == C.sizeof(P)
    assert int(out[1]) == P.rho_l.offset
    assert int(out[2]) == P.T_substrate.offset
    assert int(out[3]) == P.thermal_bc.offset
    assert int(out[4]) == P.mrt.offset and int(out[5]) == P.s_q.offset
    assert int(out[6]) == P.check_every.offset
    assert int(out[7]) == P.phi_src_mdot.offset


def test_params3_layout_matches_header(tmp_path):
    src = tmp_path / "sz3.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbf3.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(lbf3_params),'
                   ' offsetof(lbf3_params, rho_l), offsetof(lbf3_params, pcm_floor),'
                   ' offsetof(lbf3_params, wall_T), offsetof(lbf3_params, phi_src_mdot));'
                   'return 0;}\n')
    exe = tmp_path / "sz3"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    P = lbf.Params3
    assert [int(v) for v in out] == [C.sizeof(P), P.rho_l.offset, P.pcm_floor.offset,
                                     P.wall_T.offset, P.phi_src_mdot.offset]


@pytest.mark.parametrize("rb", [0, 1, 2, 4, 8, 16, 32])
def test_workspace_bytes(L, rb):
    assert L.lbf_workspace_bytes(0, 5, 0, rb) == 0
    for bad in (-64, 32, 65536 + 64):
        assert L.lbf_workspace_bytes(64, 48, bad, rb) == 0
    assert L.lbf_workspace_bytes(64, 48, 64, rb) > L.lbf_workspace_bytes(64, 48, 0, rb)
    assert L.lbf_tape_bytes(64, 48, 32, 100, 0) == 0
    assert L.lbf_tape_bytes(64, 48, 128, 100, 0) > L.lbf_tape_bytes(64, 48, 0, 100, 0)
    small = L.lbf_workspace_bytes(64, 48, 0, rb)
    big = L.lbf_workspace_bytes(2048, 2048, 0, rb)
    assert small > 64 * 48 * 4 * (27 * 2 + 9 * 2 + 4)
    # 76 resident state planes (27 + 9 ping-pong, 4 static; in row blocks
    # the static array spans the blocks' stride, 36 plane slots) + 13
    # read-out planes + reduction scratch
    lo, hi = (89, 92) if rb == 0 else (2 * 36 + 36 + 13 - 32 + 1, 2 * 36 + 36 + 13 + 3)
    assert 2048 * 2048 * 4 * lo <= big <= 2048 * 2048 * 4 * hi, big / (2048 * 2048 * 4)


def test_row_block_validation(L):
    for bad in (-1, 3, 5, 64):
        assert L.lbf_workspace_bytes(64, 48, 0, bad) == 0
        p = lbf.make_params(W.sessile_drop(nx=16, ny=8))
        p.row_block = bad
        h = C.c_void_p()
        assert L.lbf_create(C.byref(p), None, None, 0, C.byref(h)) == -1
        assert "row_block" in L.lbf_last_error().decode()
    # row blocks: a whole state array within 32-bit offsets (about 29.8 M nodes)
    assert L.lbf_workspace_bytes(4096, 4096, 0, 4) > 0
    assert L.lbf_workspace_bytes(8192, 4096, 0, 4) == 0
    assert L.lbf_workspace_bytes(8192, 4096, 0, 0) > 0        # plane-major: 27 planes


def _create_rc(L, case):
    p = lbf.make_params(case)
    p.check_every = getattr(case, "check_every", 0)
    h = C.c_void_p()
    rc = L.lbf_create(C.byref(p), None, None, 0, C.byref(h))
    return rc, L.lbf_last_error().decode()


@pytest.mark.parametrize("mutate,needle", [
    (lambda c: setattr(c, "nx", 0), "lattice size"),
    (lambda c: setattr(c.mat, "rho_ref", 1.0), "unstable"),
    (lambda c: setattr(c.mat, "mu_g", 0.0), "positive"),
    (lambda c: setattr(c.mat, "eps", -4.0), "positive"),
    (lambda c: setattr(c.mat, "pcm_floor", 1.0), "pcm_floor"),
    (lambda c: setattr(c, "thermal_bc", [2, 0, 0, 0]), "thermal_bc"),
    (lambda c: (setattr(c.mat, "mrt", 1), setattr(c.mat, "s_b", 2.0)), "MRT rates"),
    (lambda c: (setattr(c.mat, "mrt", 1), setattr(c.mat, "s_q", -0.1)), "MRT rates"),
    (lambda c: setattr(c.mat, "mrt", 2), "mrt = 2"),
    (lambda c: (setattr(c.mat, "mrt", 1), setattr(c.mat, "s_g", 2.5)), "MRT rates"),
    (lambda c: setattr(c.mat, "g_x", float("nan")), "finite"),
    (lambda c: setattr(c, "check_every", -1), "check_every"),
    (lambda c: setattr(c.mat, "phi_src_mdot", 2), "phi_src_mdot"),
])
def test_invalid_params_rejected_on_host(L, mutate, needle):
    case = W.sessile_drop(nx=16, ny=8)
    mutate(case)
    rc, msg = _create_rc(L, case)
    assert rc == -1 and needle in msg


@pytest.mark.parametrize("pad", [-64, 96, 65600])
def test_invalid_plane_pad_rejected_on_host(L, pad):
    p = lbf.make_params(W.sessile_drop(nx=16, ny=8))
    p.plane_pad = pad
    h = C.c_void_p()
    assert L.lbf_create(C.byref(p), None, None, 0, C.byref(h)) == -1
    assert "plane_pad" in L.lbf_last_error().decode()
    lbf._declare3(L)
    p3 = lbf.make_params3(W3.sphere_drop(8, 2.0))
    p3.plane_pad = pad
    assert L.lbf3_create(C.byref(p3), None, None, 0, C.byref(h)) == -1
    assert "plane_pad" in L.lbf_last_error().decode()


def test_null_arguments(L):
    assert L.lbf_step(None, 1) == -1
    assert L.lbf_reduce(None, None) == -1
    assert L.lbf_read_field(None, 0, None, 0) == -1
    L.lbf_destroy(None)
    out = C.c_void_p()
    assert L.lbf_batch_create(None, 0, C.byref(out)) == -1
    assert L.lbf_batch_step(None, 1) == -1
    assert L.lbf_batch_set_tile(None, 64, 8) == -1
    L.lbf_batch_destroy(None)
    lbf._declare3(L)
    assert L.lbf3_step(None, 1) == -1
    assert L.lbf3_reduce(None, None) == -1
    assert L.lbf3_read_fields(None, None, 0) == -1
    assert L.lbf3_set_geometry(None, None, None, 0) == -1
    assert L.lbf3_create(None, None, None, 0, C.byref(out)) == -1
    assert L.lbf3_state_bytes(None) == 0
    assert L.lbf3_save_state(None, None, 0) == -1
    assert L.lbf3_load_state(None, None, 0) == -1
    L.lbf3_destroy(None)


@pytest.mark.parametrize("rb", [0, 1, 4, 16, 64])
def test_workspace3_bytes_and_limits(L, rb):
    lbf._declare3(L)
    assert L.lbf3_workspace_bytes(0, 4, 4, 0, rb) == 0
    assert L.lbf3_workspace_bytes(4, 4, -1, 0, rb) == 0
    for bad in (-64, 32, 65536 + 64):
        assert L.lbf3_workspace_bytes(4, 4, 4, bad, rb) == 0
    assert L.lbf3_workspace_bytes(16, 16, 16, 64, rb) > L.lbf3_workspace_bytes(16, 16, 16, 0, rb)
    a, b = L.lbf3_workspace_bytes(16, 16, 16, 0, rb), L.lbf3_workspace_bytes(32, 32, 32, 0, rb)
    assert 0 < a < b
    assert L.lbf3_workspace_bytes(1024, 1024, 1024, 0, rb) == 0      # above the addressing limit
    assert L.lbf3_workspace_bytes(256, 256, 256, 0, rb) > 0           # the benchmark box
    if rb == 0:
        kmax = (0xFFFFFFFF // (4 * 19)) // 64 * 64             # nodes addressable per block
        assert L.lbf3_workspace_bytes(kmax - 64, 1, 1, 64, 0) > 0
        assert L.lbf3_workspace_bytes(kmax - 64, 1, 1, 128, 0) == 0  # the pad counts against it
    else:
        # row blocks: one f, g or h array within 32-bit offsets (its block
        # stride a power of two: 260 x 400 x 400 fits plane-major, not here)
        assert L.lbf3_workspace_bytes(260, 400, 400, 0, rb) == 0
        assert L.lbf3_workspace_bytes(260, 400, 400, 0, 0) > 0
    for bad in (-1, 3, 128):
        assert L.lbf3_workspace_bytes(16, 16, 16, 0, bad) == 0


@pytest.mark.parametrize("mutate, needle", [
    (lambda c: setattr(c, "nz", 0), "lattice size"),
    (lambda c: setattr(c.mat, "pcm_floor", 1.0), "pcm_floor"),
    (lambda c: setattr(c, "thermal_bc", [0, 0, 0, 0, 3, 0]), "thermal_bc[4]"),
    (lambda c: setattr(c.mat, "latent", -1.0), "non-negative"),
])
def test_invalid_params3_rejected_on_host(L, mutate, needle):
    from paper_2510_18688_amd import workloads3 as W3
    lbf._declare3(L)
    case = W3.sessile_drop3(nx=12, ny=10, nz=12, radius=4.0, h_s=3.0)
    mutate(case)
    p = lbf.make_params3(case)
    h = C.c_void_p()
    rc = L.lbf3_create(C.byref(p), None, None, 0, C.byref(h))
    assert rc == -1 and needle in L.lbf_last_error().decode()


def test_binding_refuses_without_device(monkeypatch):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(RuntimeError, match="HIP device"):
        lbf.Sim(W.sessile_drop(nx=16, ny=8))


def test_ch_params_layout_matches_header(tmp_path):
    from paper_2510_18688_amd import porous
    src = tmp_path / "szch.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbf_pre.h"\n'
                   'int main(void){printf("%zu %zu %zu\\n", sizeof(lbf_ch_params),'
                   ' offsetof(lbf_ch_params, A), offsetof(lbf_ch_params, dt));return 0;}\n')
    exe = tmp_path / "szch"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    P = porous.ChParams
    assert [int(v) for v in out] == [C.sizeof(P), P.A.offset, P.dt.offset]


@pytest.mark.parametrize("change, needle", [
    (dict(nx=0), "image size"),
    (dict(dt=0.05), "stability bound"),
    (dict(kappa=-1.0), "A, kappa, mobility"),
    (dict(dt=float("nan")), "A, kappa, mobility"),
])
def test_ch_invalid_params_rejected_on_host(L, change, needle):
    from paper_2510_18688_amd import porous
    porous._declare(L)
    p = porous.ch_params((8, 8), (False, False))
    for k, v in change.items():
        setattr(p, k, v)
    buf = (C.c_uint8 * 64)()
    out = (C.c_float * 64)()
    rc = L.lbf_ch_smooth(C.byref(p), buf, 0, out, 0, 1, None, None, 0)
    assert rc == -1 and needle in L.lbf_last_error().decode()
    assert L.lbf_ch_smooth(C.byref(p), None, 0, out, 0, 1, None, None, 0) == -1
    assert L.lbf_ch_workspace_bytes(0, 1, 1) == 0
    assert L.lbf_ch_workspace_bytes(65536, 65536, 1) == 0
    assert L.lbf_ch_workspace_bytes(10, 10, 1) == 2 * 512


def test_last_error_is_per_thread(L):
    """lbf_last_error() reports the calling thread's last failure: a failure
    in another thread leaves this thread's text unchanged."""
    import threading
    case = W.sessile_drop(nx=16, ny=8)
    case.nx = 0
    rc, msg = _create_rc(L, case)
    assert rc == -1 and "lattice size" in msg
    other = {}

    def worker():
        c2 = W.sessile_drop(nx=16, ny=8)
        c2.mat.pcm_floor = 1.0
        other["rc"], other["msg"] = _create_rc(L, c2)

    t = threading.Thread(target=worker)
    t.start()
    t.join()
    assert other["rc"] == -1 and "pcm_floor" in other["msg"]
    assert "lattice size" in L.lbf_last_error().decode()


def test_ch_noalloc_refuses_on_host(L):
    """The allocation-free smoothing validates like lbf_ch_smooth and
    refuses images above its stated maximum before any device call."""
    from paper_2510_18688_amd import porous
    porous._declare(L)
    n_max = L.lbf_ch_noalloc_max_nodes()
    assert n_max == 1 << 22
    out = (C.c_float * 4)(3.0, 3.0, 3.0, 3.0)
    buf = (C.c_uint8 * 4)()
    p = porous.ch_params((2, 2, n_max // 4 + 1), (True, True, True))
    rc = L.lbf_ch_smooth_noalloc(C.byref(p), buf, out, 1, None)
    assert rc == -1 and "allocation-free limit" in L.lbf_last_error().decode()
    p = porous.ch_params((8, 8), (False, False))
    p.dt = 0.05
    rc = L.lbf_ch_smooth_noalloc(C.byref(p), buf, out, 1, None)
    assert rc == -1 and "stability bound" in L.lbf_last_error().decode()
    assert L.lbf_ch_smooth_noalloc(C.byref(p), None, out, 1, None) == -1
    assert L.lbf_ch_smooth_noalloc(None, buf, out, 1, None) == -1
    assert list(out) == [3.0, 3.0, 3.0, 3.0]
