"""Parity at the benchmark sizes, in the launch configuration bench.py times
(needs a device).

Each workload runs on the GPU with the tile shape and plane padding bench.py
would pick (the autotuner's table) and on the FP64 oracle over the whole lattice, and every
read-out field is compared element by element: the O(1) fields (phi, T,
fractions, enthalpy, density) to an absolute bar, the small dynamic fields
(u, p, mu_phi) to 1e-4 of their own scale.  The batch is checked on three
sampled lattices of the 64-lattice workload after batched steps.
"""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ["phi", "T", "fl", "fs", "ux", "uy", "p", "rhoH", "mu", "C", "chi", "rho", "phihat"]
UNIT = {"phi", "T", "fl", "fs", "rhoH", "C", "chi", "rho", "phihat"}


@pytest.fixture(scope="module")
def lbf_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2510_18688_amd import lbf
    lbf.load()
    return lbf


def compare(gpu, orc, tol, label):
    worst = {}
    for k in FIELDS:
        g = gpu[k].astype(np.float64)
        o = orc[k]
        err = float(np.abs(g - o).max())
        bound = tol if k in UNIT else 1e-4 * float(np.abs(o).max()) + 1e-8
        worst[k] = err
        assert err <= bound, (label, k, err, bound)
    print(label, {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    return worst


def run_pair(lbf, oracle_mod, case, steps):
    from paper_2510_18688_amd import autotune
    tile = autotune.lookup(case.nx, case.ny)
    rb, pad = autotune.lookup_layout(case.nx, case.ny)
    sim = lbf.Sim(case, tile=tile, plane_pad=pad, row_block=rb)
    orc = oracle_mod.Oracle(case)
    sim.step(steps)
    orc.step(steps)
    return sim, orc, tile


@pytest.mark.parametrize("make", [W.curved_substrate, W.porous_medium],
                         ids=["curved_substrate_2048x2048", "porous_4096x2048"])
def test_benchmark_lattice_against_oracle(lbf_mod, oracle_mod, make):
    case = make()
    sim, orc, tile = run_pair(lbf_mod, oracle_mod, case, 20)
    print(case.name, "tile", tile, flush=True)
    compare(sim.fields(), orc.fields(), 2e-5, f"{case.name} step 20")
    # global sums of the FP64 reductions; the ice sum gathers the mushy
    # nodes along the cold wall (a few thousand, each within the 2e-5 field
    # bar), so it is held to 1e-5 of itself
    r = sim.reduce()
    ro = orc.reduce()
    for k, rel in (("sum_g", 1e-6), ("sum_h", 1e-6), ("sum_fs", 1e-5)):
        assert abs(r[k] - ro[k]) <= rel * max(abs(ro[k]), 1.0), (k, r[k], ro[k])


@pytest.mark.parametrize("make, steps", [(W.curved_substrate, 600), (W.porous_medium, 200)],
                         ids=["curved_substrate_2048x2048_600", "porous_4096x2048_200"])
def test_long_run_full_size(lbf_mod, oracle_mod, make, steps):
    """The benchmark workloads in the benchmark's configuration over many
    steps: no drift from the oracle at full size."""
    case = make()
    sim, orc, tile = run_pair(lbf_mod, oracle_mod, case, steps)
    worst = compare(sim.fields(), orc.fields(), 2e-5, f"{case.name} step {steps}")
    assert worst["phi"] <= 2e-5 and worst["fl"] <= 2e-5


def test_batched_lattices_against_oracle(lbf_mod, oracle_mod):
    from paper_2510_18688_amd import autotune
    cases = W.batch_instances(64, seed=4)
    sims = [lbf_mod.Sim(c) for c in cases]
    tile = autotune.lookup_batch(len(cases), sum(c.nodes for c in cases)) or (128, 32)
    batch = lbf_mod.Batch(sims, tile=tile)
    steps = 200
    batch.step(steps)
    picks = np.random.default_rng(7).choice(len(cases), 3, replace=False)
    for i in picks:
        orc = oracle_mod.Oracle(cases[i])
        orc.step(steps)
        compare(sims[i].fields(), orc.fields(), 2e-5, f"batch tile {tile} {cases[i].name}")


def test_gradient_workload_forward_2000_steps(lbf_mod, oracle_mod):
    """The 256 x 256 gradient workload's forward run (base controls)."""
    case, _, _ = W.adjoint_case()
    sim, orc, tile = run_pair(lbf_mod, oracle_mod, case, case.steps)
    g, o = sim.fields(), orc.fields()
    errs = {k: float(np.abs(g[k].astype(np.float64) - o[k]).max()) for k in ("phi", "T", "fl")}
    print(case.name, "tile", tile, "step", case.steps, errs, flush=True)
    for k, e in errs.items():
        assert e <= 1e-4, (k, e)
