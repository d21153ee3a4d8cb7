"""What the PCM floor (reading R45) does, checked on the FP64 oracle (no GPU).

Sec. 2 assumes that the gas takes no part in the phase change.  Read
literally (R1 with no floor), every node whose liquid weight C is positive
holds phase-change material, and gas whose phi sits a round-off above -1
near a cold wall then freezes a little: after 3000 steps of the 128 x 96
sessile freezing drop about ten thousand gas nodes (C < 0.005) hold ice, and
storing the state in FP32 moves the ice field by 4e-5.  With the floor
(C' = (C - c0)/(1 - c0), c0 = 0.01) no gas node holds ice, the FP32-storage
sensitivity of the ice field falls twenty-fold, and the frozen volume depends
on the floor's value only weakly.  The value 0.01 itself is not printed by
the paper (parity unpinned); these checks pin what it is for.
"""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W

STEPS = 3000


def _run(oracle_mod, floor, f32=False):
    case = W.sessile_drop()
    case.mat.pcm_floor = floor
    o = oracle_mod.Oracle(case)
    if f32:
        o.set_store_f32(True)
    o.step(STEPS)
    return o.fields()


@pytest.fixture(scope="module")
def runs(oracle_mod):
    return {fl: _run(oracle_mod, fl) for fl in (0.0, 0.005, 0.01, 0.02)}


def test_without_the_floor_the_gas_freezes(runs):
    F = runs[0.0]
    gas = F["C"] < 0.005
    assert int((gas & (F["fs"] > 1e-9)).sum()) > 1000
    G = runs[0.01]
    gas = G["C"] < 0.005
    assert int((gas & (G["fs"] > 0.0)).sum()) == 0


def test_floor_conditions_the_ice_field(oracle_mod, runs):
    d0 = float(np.abs(runs[0.0]["fs"] - _run(oracle_mod, 0.0, f32=True)["fs"]).max())
    d1 = float(np.abs(runs[0.01]["fs"] - _run(oracle_mod, 0.01, f32=True)["fs"]).max())
    assert d0 > 10 * d1, (d0, d1)
    assert d1 < 1e-5


def test_frozen_volume_insensitive_to_the_floor_value(runs):
    v = {fl: float(runs[fl]["fs"].sum()) for fl in (0.005, 0.01, 0.02)}
    assert abs(v[0.005] - v[0.02]) < 0.01 * v[0.01], v
