"""GPU parity of the reading switches and of the per-node isothermal region
against the FP64 oracle (needs a device).

The default workloads run one setting of each reading; these cases run the
others on a freezing drop, so that every branch the library exports is
compared with the oracle:
* cos(psi) = 0.5: the ice-wetting terms of mu_phi (eq44) are live wherever
  ice has formed;
* latch_fs = 0: the phase-change fraction is the liquid weight alone (R3);
* h_src_tau_a = 1: the enthalpy source with the printed tau_a prefactor
  (R9), with T_m = -0.2 so that the source rho C_p T mdot is nonzero;
* pcm_floor = 0: every node with a liquid weight holds phase-change
  material (R1 literally, R45 off);
* phi_src_mdot = 1: div u of the phase-field source and recovery is the
  mass source mdot (R12) instead of the flow's own divergence of the
  previous step (R54);
* a per-node isothermal region that is not phi0 >= 1/2: two patches at
  their own temperatures, one cold inside the drop and one warm in the gas.
Bars as in test_gpu_parity: 2e-6 after one step on O(1) fields, 2e-5 after
50 steps, 1e-4 after 400 steps (phi, T, f_l); small fields to 1e-4 of their
scale.
"""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W
from test_gpu_parity import FIELDS, compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbf_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2510_18688_amd import lbf
    lbf.load()
    return lbf


def _base():
    return W.slab_drop(77, 45, 13.0, 60.0, -1.5)


def _switch_cases():
    out = {}
    c = _base()
    c.mat.cos_psi = 0.5
    out["cos_psi_0.5"] = c
    c = _base()
    c.mat.latch_fs = 0
    out["latch_off"] = c
    c = _base()
    c.mat.h_src_tau_a = 1
    c.mat.T_m = -0.2
    out["h_src_tau_a"] = c
    c = _base()
    c.mat.pcm_floor = 0.0
    out["pcm_floor_0"] = c
    c = _base()
    c.mat.phi_src_mdot = 1
    out["phi_src_mdot"] = c
    c = _base()
    ny, nx = c.ny, c.nx
    hold = np.full((ny, nx), np.nan)
    hold[12:18, 30:36] = -0.7          # inside the drop, above the slab
    hold[35:40, 5:12] = 0.4            # in the gas
    c.T_hold = hold
    out["isothermal_patches"] = c
    return out


@pytest.mark.parametrize("name", list(_switch_cases()))
def test_switch_parity(lbf_mod, oracle_mod, name):
    case = _switch_cases()[name]
    sim = lbf_mod.Sim(case)
    orc = oracle_mod.Oracle(case)
    compare(sim.fields(), orc.fields(), FIELDS, 2e-6, name + " init")
    sim.step(1)
    orc.step(1)
    compare(sim.fields(), orc.fields(), FIELDS, 2e-6, name + " step 1")
    sim.step(49)
    orc.step(49)
    compare(sim.fields(), orc.fields(), ["phi", "T", "fl", "fs", "rhoH", "C", "chi"], 2e-5,
            name + " step 50")
    sim.step(350)
    orc.step(350)
    g, o = sim.fields(), orc.fields()
    compare(g, o, ["phi", "T", "fl"], 1e-4, name + " step 400")
    # the switched branch is exercised: ice has formed
    assert o["fs"].max() > 0.5, name
    gr, orr = sim.reduce(), orc.reduce()
    for k in ("sum_g", "sum_h", "sum_fs", "src_heat", "wall_flux", "reset"):
        assert abs(gr[k] - orr[k]) <= 1e-5 * max(1.0, abs(orr[k])), (name, k, gr[k], orr[k])


def test_isothermal_patches_are_held(lbf_mod):
    """The per-node region holds its own temperatures (cold patch frozen,
    warm patch liquid-free gas at 0.4), replaces the phi0 rule, and is
    removed again by a NULL mask."""
    case = _switch_cases()["isothermal_patches"]
    sim = lbf_mod.Sim(case)
    sim.step(200)
    F = sim.fields()
    inner_cold = (slice(13, 17), slice(31, 35))
    inner_warm = (slice(36, 39), slice(6, 11))
    assert np.abs(F["T"][inner_cold] + 0.7).max() < 1e-3
    assert np.abs(F["T"][inner_warm] - 0.4).max() < 1e-3
    assert F["fs"][inner_cold].min() > 0.5
    # without the region the patch is free again and warms towards the drop
    sim.set_isothermal(None, None)
    sim.step(200)
    G = sim.fields()
    assert np.abs(G["T"][inner_warm] - 0.4).max() > 1e-2


def test_isothermal_region_refused_by_the_adjoint(lbf_mod):
    case = _switch_cases()["isothermal_patches"]
    sim = lbf_mod.Sim(case)
    with pytest.raises(lbf_mod.LbfError, match="per-node isothermal"):
        lbf_mod.Tape(sim, 10)


def test_flow_divergence_source_refused_by_the_adjoint(lbf_mod):
    case = _base()
    assert case.mat.phi_src_mdot == 0
    sim = lbf_mod.Sim(case)
    with pytest.raises(lbf_mod.LbfError, match="phi_src_mdot"):
        lbf_mod.Tape(sim, 10)
