"""The state's memory layout (lbf_params.row_block: plane-major, or row
blocks of 1 .. 32 rows holding every plane of those rows) is a layout choice
only (needs a device): in every layout the step, the read-out, the
reductions, the observables, the isothermal region, a state set from
outside, the checkpoint and the batched launch give the same bits, on
lattices whose height is not a multiple of the block, and a checkpoint moves
between layouts."""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ["phi", "T", "fl", "fs", "ux", "uy", "p", "rhoH", "mu", "C", "chi", "rho", "phihat"]
LAYOUTS = [1, 2, 4, 8, 16, 32]


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


CASES = {
    # ny 61: a partial last block for every block height above 1
    "porous_ragged_147x61": lambda: W.porous_medium(nx=147, ny=61, seed=5, rmin=6.0, rmax=10.0,
                                                    porosity=0.8),
    "sessile_64x45": lambda: W.sessile_drop(nx=64, ny=45, radius=12.0),
    "cylinder_mdot_96": lambda: _mdot(W.curved_substrate(n=96, R_s=20.0, R_0=15.0)),
}


def _mdot(case):
    case.mat.phi_src_mdot = 1
    return case


@pytest.mark.parametrize("rb", LAYOUTS)
@pytest.mark.parametrize("name", sorted(CASES))
def test_layout_gives_the_same_bits(lbf_mod, rb, name):
    a = lbf_mod.Sim(CASES[name](), row_block=0)
    b = lbf_mod.Sim(CASES[name](), row_block=rb, plane_pad=64)
    for tile in ((64, 3), (256, 16)):
        a.set_tile(*tile)
        b.set_tile(*tile)
        a.step(37)
        b.step(37)
        same(a.fields(), b.fields(), f"{name} row_block {rb} tile {tile}")
    ra, rbd = a.reduce(), b.reduce()
    for k in ra:
        assert ra[k] == rbd[k] or (np.isnan(ra[k]) and np.isnan(rbd[k])), k
    pa, pb = a.profiles(), b.profiles()
    for part in ("col", "row"):
        for k in pa[part]:
            assert np.array_equal(pa[part][k], pb[part][k]), (part, k)


@pytest.mark.parametrize("phi_src_mdot", [0, 1])
def test_layout_with_isothermal_region_and_outside_state(lbf_mod, phi_src_mdot):
    case = lambda: W.sessile_drop(nx=90, ny=53, radius=14.0)
    sims = []
    for rb in (0, 4, 8):
        c = case()
        c.mat.phi_src_mdot = phi_src_mdot
        s = lbf_mod.Sim(c, row_block=rb)
        mask = np.zeros((c.ny, c.nx), dtype=bool)
        mask[:9, 20:70] = True
        s.set_isothermal(mask, np.full((c.ny, c.nx), c.mat.T_m - 0.3))
        s.init_fields(c.phi, c.T)
        s.step(25)
        sims.append(s)
    for s in sims[1:]:
        same(sims[0].fields(), s.fields(), "isothermal")
    # a post-stream state set from outside (the layout the caller sees is
    # plane-major in every case)
    rng = np.random.default_rng(3)
    c = case()
    c.mat.phi_src_mdot = phi_src_mdot
    n = c.nx * c.ny
    dist = (rng.standard_normal((27, n)) * 1e-3).astype(np.float32)
    dist[9] += 1.0
    dist[18] += 1.0
    lag = np.zeros((7, n), dtype=np.float32)
    lag[0] = rng.uniform(0.0, 0.2, n)
    outs = []
    for rb in (0, 2, 16):
        s = lbf_mod.Sim(c, row_block=rb)
        s.set_poststream_state(dist[:9], dist[9:18], dist[18:], lag, 5)
        s.step(3)
        outs.append(s.fields())
    for o in outs[1:]:
        same(outs[0], o, "outside state")


def test_checkpoint_moves_between_layouts(lbf_mod):
    import torch
    case = lambda: W.porous_medium(nx=131, ny=67, seed=5, rmin=6.0, rmax=10.0, porosity=0.8)
    a, b = lbf_mod.Sim(case(), row_block=0), lbf_mod.Sim(case(), row_block=4, plane_pad=128)
    assert a.state_bytes() == b.state_bytes() == (27 + 9) * 131 * 67 * 4 + 64
    a.step(25)
    buf = torch.empty(a.state_bytes(), dtype=torch.uint8, device="cuda")
    a.save_state(buf)
    b.load_state(buf)
    a.step(15)
    b.step(15)
    same(a.fields(), b.fields(), "checkpoint plane-major -> 4-row blocks")
    b.save_state(buf)
    c = lbf_mod.Sim(case(), row_block=32)
    c.load_state(buf)
    c.step(5)
    a.step(5)
    same(a.fields(), c.fields(), "checkpoint 4-row -> 32-row blocks")
    # the saved bytes do not depend on the layout
    buf2 = torch.empty_like(buf)
    a.save_state(buf)
    c.save_state(buf2)
    assert torch.equal(buf, buf2)


def test_layout_batch_and_full_size(lbf_mod):
    cases = W.batch_instances(count=5, seed=9, lo=40, hi=120)
    ref = [lbf_mod.Sim(c, row_block=0) for c in cases]
    for s in ref:
        s.step(30)
    sims = [lbf_mod.Sim(c, row_block=[1, 2, 4, 8, 16][i]) for i, c in enumerate(cases)]
    lbf_mod.Batch(sims, tile=(128, 8)).step(30)
    for r, s in zip(ref, sims):
        same(r.fields(), s.fields(), s.case.name)
    case = W.curved_substrate()
    a = lbf_mod.Sim(case, tile=(256, 16), row_block=0, plane_pad=576)
    b = lbf_mod.Sim(case, tile=(256, 16), row_block=4, plane_pad=64)
    a.step(12)
    b.step(12)
    same(a.fields(), b.fields(), "2048^2 4-row blocks")
    ma, ba = a.copy_probe(3)
    mb, bb = b.copy_probe(3)
    assert ba == bb
    a.step(3)
    b.step(3)
    same(a.fields(), b.fields(), "2048^2 after the copy probe")


def test_adjoint_needs_plane_major(lbf_mod):
    sim = lbf_mod.Sim(W.small_freezing_case(), row_block=4)
    with pytest.raises(lbf_mod.LbfError, match="row_block"):
        lbf_mod.Tape(sim, 10)
