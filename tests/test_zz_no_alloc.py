"""The allocation-free smoothing entry point (lbf_ch_smooth_noalloc),
called through the C ABI, against the allocating one (lbf_ch_smooth) on the
same device images: two calls in a row, the second on a smaller image, both
bit for bit (the two share their kernels; only where the working planes
live differs).  Also: images above the stated maximum are refused before any
device work."""

import ctypes as C

import numpy as np
import pytest

from paper_2510_18688_amd import lbf, porous, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    L = lbf.load()
    porous._declare(L)
    return L


def _both(L, img, periodic, iterations):
    """phi0 from the allocating entry point (library-owned workspace) and
    from the allocation-free one, both on device buffers and one stream."""
    import torch
    solid = torch.from_numpy(np.ascontiguousarray(img != 0, dtype=np.uint8)).cuda()
    ref = torch.full(img.shape, -7.0, dtype=torch.float32, device="cuda")
    out = torch.full(img.shape, -7.0, dtype=torch.float32, device="cuda")
    p = porous.ch_params(img.shape, periodic)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.lbf_ch_smooth(C.byref(p), C.c_void_p(solid.data_ptr()), 1, C.c_void_p(ref.data_ptr()),
                         1, iterations, st, None, 0)
    assert rc == 0, L.lbf_last_error().decode()
    rc = L.lbf_ch_smooth_noalloc(C.byref(p), C.c_void_p(solid.data_ptr()),
                                 C.c_void_p(out.data_ptr()), iterations, st)
    assert rc == 0, L.lbf_last_error().decode()
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_matches_allocating_entry_point_twice(L):
    print("case: 2D 700 x 500 sandpack, walls, 120 steps; then 3D 37 x 29 x 23, 60 steps",
          flush=True)
    big = W.sandpack_image((500, 700), seed=11, r_median=9.0)
    ref, out = _both(L, big, (False, False), 120)
    assert np.isfinite(ref).all() and ref.min() >= 0.0 and ref.max() <= 1.0
    assert np.array_equal(ref, out)
    rng = np.random.default_rng(12)
    small = (rng.random((23, 29, 37)) < 0.4).astype(np.uint8)
    ref2, out2 = _both(L, small, (True, False, True), 60)
    assert np.isfinite(ref2).all()
    assert np.array_equal(ref2, out2)
    # the second call left no trace of the first's larger image
    ref3, out3 = _both(L, small[:, :11, :13].copy(), (False, True, False), 7)
    assert np.array_equal(ref3, out3)


def test_noalloc_matches_the_binding_and_refuses_large_images(L):
    import torch
    n_max = L.lbf_ch_noalloc_max_nodes()
    assert n_max == 1 << 22
    img = W.sandpack_image((64, 96), seed=3, r_median=5.0)
    solid = torch.from_numpy(np.ascontiguousarray(img != 0, dtype=np.uint8)).cuda()
    out = torch.empty(img.shape, dtype=torch.float32, device="cuda")
    got = porous.ch_smooth_noalloc(solid, out, (True, False), 40).cpu().numpy()
    want = porous.ch_smooth(img, (True, False), 40)
    assert np.array_equal(got, want)
    # one node over the limit: refused on the host, the output untouched
    p = porous.ch_params((1, 1, n_max + 1), (True, True, True))
    out.fill_(3.0)
    rc = L.lbf_ch_smooth_noalloc(C.byref(p), C.c_void_p(solid.data_ptr()),
                                 C.c_void_p(out.data_ptr()), 1, None)
    assert rc == -1 and "allocation-free limit" in L.lbf_last_error().decode()
    assert L.lbf_ch_smooth_noalloc(C.byref(p), None, C.c_void_p(out.data_ptr()), 1, None) == -1
    torch.cuda.synchronize()
    assert float(out.min()) == 3.0 == float(out.max())
