"""Batched persistent launch (needs a device): every lattice of a batch is
advanced exactly as lbf_step advances it, whatever the tile shape, the
number of steps (graph replays and direct launches) or individual steps in
between."""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbf_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2510_18688_amd import lbf
    lbf.load()
    return lbf


def uneven_cases():
    cases = W.batch_instances(count=6, seed=4, lo=40, hi=150)
    cases.append(W.curved_substrate(n=96, R_s=20.0, R_0=15.0))
    cases.append(W.porous_medium(nx=130, ny=70, seed=11, rmin=8.0, rmax=12.0, porosity=0.8))
    return cases


@pytest.mark.parametrize("tile,steps", [((64, 8), 5), ((128, 32), 37), ((256, 16), 70)])
def test_batch_matches_single_lattice_steps(lbf_mod, tile, steps):
    cases = uneven_cases()
    singles = [lbf_mod.Sim(c) for c in cases]
    for s in singles:
        s.step(steps)
    ref = [s.fields() for s in singles]
    sims = [lbf_mod.Sim(c) for c in cases]
    batch = lbf_mod.Batch(sims, tile=tile)
    batch.step(steps)
    assert batch.items() > len(cases)
    for r, s in zip(ref, sims):
        got = s.fields()
        for k in ("phi", "T", "fs", "ux", "p", "rhoH"):
            assert np.array_equal(r[k], got[k]), (s.case.name, k)
        assert s.reduce()["step"] == steps


def test_batch_interleaved_with_single_steps(lbf_mod):
    cases = uneven_cases()[:4]
    ref = [lbf_mod.Sim(c) for c in cases]
    for s in ref:
        s.step(3 + 33 + 2)
    sims = [lbf_mod.Sim(c) for c in cases]
    batch = lbf_mod.Batch(sims, tile=(128, 16))
    batch.step(3)
    sims[1].step(33)          # one lattice moves on its own
    for i in (0, 2, 3):
        sims[i].step(33)
    batch.step(2)
    for r, s in zip(ref, sims):
        a, b = r.fields(), s.fields()
        for k in ("phi", "T", "fs", "p"):
            assert np.array_equal(a[k], b[k]), (s.case.name, k)


def test_batch_rejects_mixed_streams(lbf_mod):
    import torch
    a = lbf_mod.Sim(W.sessile_drop(nx=32, ny=16))
    other = torch.cuda.Stream()
    b = lbf_mod.Sim(W.sessile_drop(nx=32, ny=16), stream=other)
    with pytest.raises(lbf_mod.LbfError):
        lbf_mod.Batch([a, b])
    with pytest.raises(lbf_mod.LbfError):
        lbf_mod.Batch([a, a])
