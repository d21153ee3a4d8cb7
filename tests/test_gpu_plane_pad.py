"""The plane padding of the workspace (lbf_params.plane_pad) is a layout
choice only (needs a device): with any pad the step, the read-out, the
reductions, the checkpoint, the batched launch and the adjoint give the
same bits as without one, and a checkpoint moves between simulations of
different pads."""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ["phi", "T", "fl", "fs", "ux", "uy", "p", "rhoH", "mu", "C", "chi", "rho", "phihat"]


@pytest.fixture(scope="module")
def lbf_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2510_18688_amd import lbf
    lbf.load()
    return lbf


def same(a, b, label):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), (label, k)


@pytest.mark.parametrize("pad", [64, 2112, 65536])
@pytest.mark.parametrize("name", ["sessile_64x48", "porous_ragged_147x61"])
def test_pad_gives_the_same_bits(lbf_mod, pad, name):
    case = {"sessile_64x48": lambda: W.sessile_drop(nx=64, ny=48, radius=15.0),
            "porous_ragged_147x61": lambda: W.porous_medium(nx=147, ny=61, seed=5, rmin=6.0,
                                                           rmax=10.0, porosity=0.8)}[name]
    a, b = lbf_mod.Sim(case()), lbf_mod.Sim(case(), plane_pad=pad)
    assert b.workspace.numel() > a.workspace.numel()
    a.step(120)
    b.step(120)
    same(a.fields(), b.fields(), f"{name} pad {pad}")
    ra, rb = a.reduce(), b.reduce()
    for k in ("sum_g", "sum_h", "sum_fs", "umax"):
        assert ra[k] == rb[k], k
    pa, pb = a.profiles(), b.profiles()
    for part in ("col", "row"):
        for k in pa[part]:
            assert np.array_equal(pa[part][k], pb[part][k]), (part, k)


def test_pad_checkpoint_and_full_size(lbf_mod):
    import torch
    from paper_2510_18688_amd import autotune
    case = W.curved_substrate()
    a = lbf_mod.Sim(case, tile=(256, 8))
    b = lbf_mod.Sim(case, tile=(256, 8), plane_pad=2112)
    a.step(20)
    b.step(20)
    same(a.fields(), b.fields(), "2048^2 pad 2112")
    buf = torch.empty(b.state_bytes(), dtype=torch.uint8, device="cuda")
    b.save_state(buf)
    b.step(5)
    b.load_state(buf)
    b.step(5)
    a.step(5)
    same(a.fields(), b.fields(), "2048^2 pad 2112 after reload")
    assert autotune.lookup_pad(2048, 2048) % 64 == 0


def test_pad_batch_and_adjoint(lbf_mod):
    cases = W.batch_instances(count=4, seed=9, lo=40, hi=120)
    ref = [lbf_mod.Sim(c) for c in cases]
    for s in ref:
        s.step(30)
    sims = [lbf_mod.Sim(c, plane_pad=64 * (i + 1)) for i, c in enumerate(cases)]
    lbf_mod.Batch(sims, tile=(128, 16)).step(30)
    for r, s in zip(ref, sims):
        same(r.fields(), s.fields(), s.case.name)
    grads = []
    for pad in (0, 4160):
        case = W.small_freezing_case()
        sim = lbf_mod.Sim(case, plane_pad=pad, row_block=0)
        tape = lbf_mod.Tape(sim, 40, 7)
        tape.forward()
        seed = np.ones((case.ny, case.nx), dtype=np.float32)
        gc, gw = tape.backward(seed_fs=seed)
        grads.append((gc.cpu().numpy(), gw.cpu().numpy()))
        tape.close()
    assert np.array_equal(grads[0][0], grads[1][0])
    assert np.array_equal(grads[0][1], grads[1][1])
    assert np.abs(grads[0][0]).max() > 0


@pytest.mark.parametrize("pad", [64, 4160])
def test_pad_gives_the_same_bits_3d(lbf_mod, pad):
    import torch
    from paper_2510_18688_amd import workloads3 as W3
    case = lambda: W3.fracture(nx=40, ny=24, nz=18, aperture=8.0, roughness=1.5)
    a, b = lbf_mod.Sim3(case()), lbf_mod.Sim3(case(), plane_pad=pad)
    a.step(40)
    b.step(40)
    Fa, Fb = a.fields(), b.fields()
    for k in Fa:
        assert np.array_equal(Fa[k], Fb[k]), k
    ra, rb = a.reduce(), b.reduce()
    for k in ("sum_g", "sum_h", "sum_fs", "umax"):
        assert ra[k] == rb[k], k
    buf = torch.empty(b.state_bytes(), dtype=torch.uint8, device="cuda")
    b.save_state(buf)
    b.step(7)
    b.load_state(buf)
    b.step(7)
    a.step(7)
    Fa, Fb = a.fields(), b.fields()
    for k in Fa:
        assert np.array_equal(Fa[k], Fb[k]), k


def test_checkpoint_moves_between_pads(lbf_mod):
    import torch
    from paper_2510_18688_amd import workloads3 as W3
    case = lambda: W.porous_medium(nx=131, ny=67, seed=5, rmin=6.0, rmax=10.0, porosity=0.8)
    a, b = lbf_mod.Sim(case()), lbf_mod.Sim(case(), plane_pad=4160)
    assert a.state_bytes() == b.state_bytes() == (27 + 9) * 131 * 67 * 4 + 64
    a.step(25)
    buf = torch.empty(a.state_bytes(), dtype=torch.uint8, device="cuda")
    a.save_state(buf)
    b.load_state(buf)
    a.step(15)
    b.step(15)
    same(a.fields(), b.fields(), "2D checkpoint pad 0 -> 4160")
    b.save_state(buf)
    c = lbf_mod.Sim(case(), plane_pad=64)
    c.load_state(buf)
    c.step(5)
    a.step(5)
    same(a.fields(), c.fields(), "2D checkpoint pad 4160 -> 64")
    case3 = lambda: W3.fracture(nx=36, ny=20, nz=14, aperture=7.0, roughness=1.5)
    d, e = lbf_mod.Sim3(case3(), plane_pad=4224), lbf_mod.Sim3(case3())
    d.step(12)
    buf3 = torch.empty(d.state_bytes(), dtype=torch.uint8, device="cuda")
    d.save_state(buf3)
    e.load_state(buf3)
    d.step(9)
    e.step(9)
    Fd, Fe = d.fields(), e.fields()
    for k in Fd:
        assert np.array_equal(Fd[k], Fe[k]), k
