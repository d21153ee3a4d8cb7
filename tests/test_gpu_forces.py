"""GPU parity of the body force G = rho g and the solid-phase velocity u_s
of the drag (needs a device): element by element against the FP64 oracles
after 1 and 300 steps on freezing 2D and 3D workloads with gravity and a
moving solid, the Couette flow of a moving slab against the oracle's, and
the adjoint's refusal."""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W, workloads3 as W3

pytestmark = pytest.mark.gpu

UNIT = {"phi", "T", "fl", "fs", "rhoH", "C", "chi", "rho", "phihat"}


@pytest.fixture(scope="module")
def lbf_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2510_18688_amd import lbf
    lbf.load()
    return lbf


def compare(gpu, orc, names, tol, label):
    worst = {}
    for k in names:
        g, o = gpu[k].astype(np.float64), orc[k]
        err = float(np.abs(g - o).max())
        bound = tol if k in UNIT else max(tol, 1e-4) * float(np.abs(o).max()) + 1e-8
        worst[k] = err
        assert err <= bound, (label, k, err, bound)
    print(label, {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)


def forced(case, **kw):
    for k, v in kw.items():
        setattr(case.mat, k, v)
    return case


CASES2 = {
    "sessile_gravity": lambda: forced(W.sessile_drop(nx=64, ny=48, radius=15.0), g_y=-2e-5),
    "slab_moving_gravity": lambda: forced(W.slab_drop(77, 45, 13.0, 60.0, -1.5), g_x=1e-5,
                                          g_y=-1e-5, us_x=2e-3),
    "porous_gravity": lambda: forced(W.porous_medium(nx=160, ny=96, seed=11, rmin=8.0, rmax=14.0,
                                                     porosity=0.8), g_x=-1e-5, us_y=1e-3),
}


@pytest.mark.parametrize("name", list(CASES2))
def test_forces_2d_match_oracle(lbf_mod, name):
    from oracle import oracle as O
    case = CASES2[name]()
    sim, orc = lbf_mod.Sim(case), O.Oracle(case)
    sim.step(1)
    orc.step(1)
    compare(sim.fields(), orc.fields(), ["phi", "T", "fs", "ux", "uy", "p", "rhoH", "mu"], 2e-6,
            f"{name} step 1")
    sim.step(299)
    orc.step(299)
    compare(sim.fields(), orc.fields(), ["phi", "T", "fl", "fs", "rhoH", "C", "chi"], 2e-5,
            f"{name} step 300")


def test_forces_3d_match_oracle(lbf_mod):
    from oracle import oracle3 as O3
    O3.build()
    case = forced(W3.sessile_drop3(nx=30, ny=26, nz=22, radius=8.0, h_s=4.0), g_z=-2e-5,
                  g_x=5e-6, us_y=1e-3)
    sim, orc = lbf_mod.Sim3(case), O3.Oracle3(case)
    sim.step(1)
    orc.step(1)
    compare(sim.fields(), orc.fields(), ["phi", "T", "fs", "ux", "uy", "uz", "p", "rhoH"], 2e-6,
            "sessile3 forced step 1")
    sim.step(99)
    orc.step(99)
    compare(sim.fields(), orc.fields(), ["phi", "T", "fl", "fs", "rhoH", "C", "chi"], 2e-5,
            "sessile3 forced step 100")


def test_moving_slab_couette_matches_oracle(lbf_mod):
    from oracle import oracle as O
    H, U = 48, 1e-3
    mat = W.Material(us_x=U)
    z = np.zeros((H, 4))
    case = W.Case("couette", 4, H, True, False, [0, 0, 0, 0], {}, W.slab_phi0(4, H, 8.0, mat.eps),
                  z.copy(), np.ones((H, 4)), np.full((H, 4), 0.5), mat)
    sim, orc = lbf_mod.Sim(case), O.Oracle(case)
    sim.step(5000)
    orc.step(5000)
    g, o = sim.fields()["ux"][:, 1], orc.fields()["ux"][:, 1]
    assert np.abs(g - o).max() < 1e-4 * U, np.abs(g - o).max() / U


def test_adjoint_refuses_forces(lbf_mod):
    case = forced(W.small_freezing_case(), g_y=-1e-5)
    sim = lbf_mod.Sim(case)
    with pytest.raises(lbf_mod.LbfError, match="grav"):
        lbf_mod.Tape(sim, 10)
