"""Behaviour of the paper's complex-geometry cases on the GPU at full size
over thousands of steps (needs a device; properties that hold at any size,
where the oracle cannot follow):

* freezing in the rough fracture (Sec. 4.5): ice forms at the cold face and
  its front advances along x; the far part of the liquid column stays
  unfrozen (but for traces at its interface with the gas: the column starts
  at the melting point); ice never exceeds the phase-change material (f_s <= chi) and the
  gas bubbles hold none;
* freezing in the prepared unsaturated porous medium (Sec. 4.6): after the
  smoothing and the phase separation, the front moves from the cold wall
  towards the warm one.
"""

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


def front(profile, level):
    """First index where a decreasing profile drops below `level`."""
    below = np.nonzero(profile < level)[0]
    return int(below[0]) if below.size else len(profile)


def test_fracture_freezing_front(lbf_mod):
    case = W3.fracture()
    sim = lbf_mod.Sim3(case)
    fronts = []
    for n in (2000, 3000):
        sim.step(n)
        F = sim.fields()
        slab = F["fs"].mean(axis=(0, 1))
        fronts.append(front(slab, 0.5 * slab[0]))
        assert slab[:10].mean() > 0.4                         # frozen at the cold face
        # far liquid: unfrozen but for traces where the liquid meets the gas
        # (the column starts at T_m, so its moving interface sits at the
        # melting point)
        assert slab[100:190].max() < 0.03
        assert float((F["fs"] - F["chi"]).max()) <= 1e-5      # ice only within the PCM
        gas = (F["phi"] < -0.95) & (case.phi0 < 0.05)
        assert gas.any() and float(F["fs"][gas].max()) < 0.03
        assert sim.reduce()["nonfinite"] == 0
    print("fracture fronts (x) after 2000 and 5000 steps:", fronts, flush=True)
    assert fronts[0] >= 15 and fronts[1] > fronts[0]


def test_porous_freezing_front(lbf_mod):
    from paper_2510_18688_amd import porous
    img = W.sandpack_image((256, 512), seed=12, r_median=6.0)
    sim, case = porous.prepare(img, S_w=0.5, theta_deg=60.0, ch_iterations=500,
                               separation_steps=3000)
    assert sim.reduce()["sum_fs"] == 0.0                      # no ice during the separation
    sim.set_wall_temperature(W.LEFT, np.full(case.ny, -1.0))
    sim.set_wall_temperature(W.RIGHT, np.full(case.ny, 0.5))
    fronts = []
    for n in (3000, 3000):
        sim.step(n)
        F = sim.fields()
        share = F["fs"].sum(axis=0) / np.maximum(F["chi"].sum(axis=0), 1e-9)
        fronts.append(front(share, 0.5))
        assert share[:10].min() > 0.9 and share[100:].max() == 0.0
    print("porous fronts (x) after 3000 and 6000 freezing steps:", fronts, flush=True)
    assert fronts[1] > fronts[0]
