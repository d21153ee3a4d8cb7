"""The D3Q19 state's memory layout (lbf3_params.row_block: plane-major, or
row blocks of 1 .. 64 rows of nx nodes holding every plane of the f, g, h,
lagged and static arrays) is a layout choice only (needs a device): every
layout gives the same bits for the step, the read-out and the reductions,
with either phase-field source, on lattices whose row count is not a
multiple of the block, at the fracture's full size, and a checkpoint moves
between layouts with identical saved bytes."""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W, workloads3 as W3

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbf_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2510_18688_amd import lbf
    lbf.load()
    return lbf


def same(a, b, label):
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(a[k], b[k]), (label, k)


CASES = {
    # 21 x 19 x 17: 323 rows, a partial last block for every block height above 1
    "boxed_ragged": lambda: W3.sessile_drop3(nx=21, ny=19, nz=17, radius=6.0, h_s=3.0),
    "fracture_small": lambda: W3.fracture(nx=40, ny=24, nz=18, aperture=8.0, roughness=1.5),
    "porous_walls_xy": lambda: W3.from_2d(W.porous_medium(nx=50, ny=34, seed=11, rmin=4.0,
                                                          rmax=6.0, porosity=0.8),
                                          axis="z", depth=5),
}


@pytest.mark.parametrize("mdot", [0, 1])
@pytest.mark.parametrize("rb", [1, 4, 16, 64])
@pytest.mark.parametrize("name", sorted(CASES))
def test_layout3_gives_the_same_bits(lbf_mod, name, rb, mdot):
    ca, cb = CASES[name](), CASES[name]()
    ca.mat.phi_src_mdot = cb.mat.phi_src_mdot = mdot
    a = lbf_mod.Sim3(ca, row_block=0)
    b = lbf_mod.Sim3(cb, row_block=rb, plane_pad=64)
    same(a.fields(), b.fields(), f"{name} rb {rb} init")
    a.step(23)
    b.step(23)
    same(a.fields(), b.fields(), f"{name} rb {rb} step 23")
    ra, rbd = a.reduce(), b.reduce()
    for k in ra:
        assert ra[k] == rbd[k], k


def test_checkpoint3_moves_between_layouts(lbf_mod):
    import torch
    case = CASES["boxed_ragged"]
    a, b = lbf_mod.Sim3(case(), row_block=16), lbf_mod.Sim3(case(), row_block=0)
    a.step(11)
    buf = torch.empty(a.state_bytes(), dtype=torch.uint8, device="cuda")
    a.save_state(buf)
    b.load_state(buf)
    a.step(9)
    b.step(9)
    same(a.fields(), b.fields(), "16-row blocks -> plane-major")
    c = lbf_mod.Sim3(case(), row_block=1, plane_pad=128)
    b.save_state(buf)
    c.load_state(buf)
    c.step(4)
    a.step(4)
    same(a.fields(), c.fields(), "plane-major -> 1-row blocks")
    buf2 = torch.empty_like(buf)
    a.save_state(buf)
    c.save_state(buf2)
    assert torch.equal(buf, buf2)


def test_layout3_full_size_fracture(lbf_mod):
    a = lbf_mod.Sim3(W3.fracture(), row_block=0, plane_pad=4224)
    b = lbf_mod.Sim3(W3.fracture(), row_block=16)
    a.step(6)
    b.step(6)
    same(a.fields(), b.fields(), "fracture 256 x 128 x 30")
