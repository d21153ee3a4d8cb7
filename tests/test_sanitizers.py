"""AddressSanitizer and UndefinedBehaviorSanitizer on the host code (no GPU).

* The FP64 oracles (2D and 3D C sources) built with
  -fsanitize=address,undefined and run through their Python wrappers on small
  workloads that reach every pass: walls on x and y with Dirichlet faces, a
  held region given per node, MRT, both phase-field sources, state save and
  restore, reductions.
* The library's host code (every .hip source, host side instrumented, device
  side compiled as usual) linked into tests/sanitize/host_driver.cpp, which
  runs the paths that need no device: sizes, parameter validation, refusals,
  NULL handles, the per-thread error text, and the failing allocation of a
  valid parameter set.
Any sanitizer finding aborts the run and fails the test.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _libasan():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracles_under_asan_and_ubsan(tmp_path):
    asan = _libasan()
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime not found")
    libs = {}
    for name, src in (("ORC2", "lbf_oracle.c"), ("ORC3", "lbf_oracle3.c")):
        out = str(tmp_path / f"lib{name}.so")
        subprocess.run(["gcc", "-O1", *SAN, "-ffp-contract=off", "-fPIC", "-shared", "-o", out,
                        os.path.join(ROOT, "oracle", src), "-lm"], check=True)
        libs["LBF_" + name] = out
    env = dict(os.environ, **libs, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run(["python3", os.path.join(ROOT, "tests", "sanitize", "oracle_run.py")],
                       env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "oracle runs clean" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2510_18688_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in ("lbf_api.hip", "lbf_adjoint.hip", "lbf_observe.hip",
                                            "lbf3_api.hip", "lbf_pre.hip")]
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f] if f.startswith("-fsanitize") or f.startswith("-fno-san") else [f]
    lib = str(tmp_path / "liblbf_san.so")
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + csrc]
    subprocess.run([HIPCC, "-O1", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-w", *host_san,
                    *inc, *srcs, "-o", lib], check=True, capture_output=True)
    exe = str(tmp_path / "host_driver")
    subprocess.run([HIPCC, "-O1", "-std=c++17", "-w", *host_san, *inc,
                    os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                    "-L" + str(tmp_path), "-llbf_san", "-Wl,-rpath," + str(tmp_path), "-o", exe],
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout
