"""GPU parity of the D3Q19 coupled step against the FP64 3D oracle (needs a
device): element by element on the same seeded inputs, after the
initialisation, one step and a few tens of steps, on lattices with periodic
axes, walls on every face, Dirichlet faces, a held substrate and ragged
sizes; the 3D workload (the rough fracture) at full size after a few steps;
and the global sums.  Bars as in the 2D parity: O(1) fields (phi, T,
fractions, enthalpy, density) to an absolute bar, the small dynamic fields
(u, p, mu_phi) to 1e-4 of their own scale."""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W, workloads3 as W3

pytestmark = pytest.mark.gpu

FIELDS3 = ["phi", "T", "fl", "fs", "ux", "uy", "uz", "p", "rhoH", "mu", "C", "chi", "rho",
           "phihat"]
UNIT = {"phi", "T", "fl", "fs", "rhoH", "C", "chi", "rho", "phihat"}


@pytest.fixture(scope="module")
def lbf_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2510_18688_amd import lbf
    lbf.load()
    return lbf


@pytest.fixture(scope="module")
def O3():
    from oracle import oracle3
    oracle3.build()
    return oracle3


def compare(gpu, orc, tol, label, names=FIELDS3):
    worst = {}
    for k in names:
        g = gpu[k].astype(np.float64)
        o = orc[k]
        err = float(np.abs(g - o).max())
        bound = tol if k in UNIT else max(tol, 1e-4) * float(np.abs(o).max()) + 1e-8
        worst[k] = err
        assert err <= bound, (label, k, err, bound)
    print(label, {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)


def boxed():
    """A drop in a closed box: walls on all six faces, three of them held at
    different temperatures, so links through edges meet two walls."""
    c = W3.sessile_drop3(nx=21, ny=19, nz=17, radius=6.0, h_s=3.0)
    c.name = "boxed_21x19x17"
    c.periodic = (False, False, False)
    c.thermal_bc = [0, 1, 1, 0, 1, 0]
    c.wall_T = [0.0, -0.6, -0.3, 0.0, -1.2, 0.0]
    return c


def cases():
    return {
        "boxed_21x19x17": boxed(),
        "sessile3_30x26x22": W3.sessile_drop3(nx=30, ny=26, nz=22, radius=8.0, h_s=4.0),
        "sphere_24": W3.sphere_drop(24, 7.0),
        "porous_walls_xy": W3.from_2d(W.porous_medium(nx=50, ny=34, seed=11, rmin=4.0, rmax=6.0,
                                                      porosity=0.8), axis="z", depth=5),
        "curved_held_y": W3.from_2d(W.curved_substrate(n=40, R_s=8.0, R_0=7.0), axis="y", depth=3),
        "fracture_small": W3.fracture(nx=40, ny=24, nz=18, aperture=8.0, roughness=1.5),
    }


@pytest.mark.parametrize("name", list(cases()))
def test_one_step_and_few_steps(lbf_mod, O3, name):
    case = cases()[name]
    sim = lbf_mod.Sim3(case)
    orc = O3.Oracle3(case)
    compare(sim.fields(), orc.fields(), 2e-6, name + " init")
    sim.step(1)
    orc.step(1)
    compare(sim.fields(), orc.fields(), 2e-6, name + " step 1")
    sim.step(29)
    orc.step(29)
    compare(sim.fields(), orc.fields(), 2e-5, name + " step 30",
            ["phi", "T", "fl", "fs", "rhoH", "C", "chi"])
    r, ro = sim.reduce(), orc.reduce()
    for k in ("sum_g", "sum_h", "sum_fs"):
        assert abs(r[k] - ro[k]) <= 1e-6 * max(abs(ro[k]), 1.0), (name, k, r[k], ro[k])


@pytest.mark.parametrize("name", ["boxed_21x19x17", "fracture_small"])
def test_mass_source_reading(lbf_mod, O3, name):
    """The phase-field source with the model's mass source as div u (R12,
    phi_src_mdot = 1: no velocity planes) against the oracle with the same
    reading."""
    case = cases()[name]
    case.mat.phi_src_mdot = 1
    sim = lbf_mod.Sim3(case)
    orc = O3.Oracle3(case)
    sim.step(1)
    orc.step(1)
    compare(sim.fields(), orc.fields(), 2e-6, name + " R12 step 1")
    sim.step(29)
    orc.step(29)
    compare(sim.fields(), orc.fields(), 2e-5, name + " R12 step 30",
            ["phi", "T", "fl", "fs", "rhoH", "C", "chi"])


def test_fracture_full_size(lbf_mod, O3):
    """The full fracture in the benchmark's configuration (its tuned plane
    padding) after 5 steps, and the freezing fields after 300."""
    from paper_2510_18688_amd import autotune
    case = W3.fracture()
    rb, pad = autotune.lookup_layout3(case.nx, case.ny, case.nz)
    sim = lbf_mod.Sim3(case, plane_pad=pad, row_block=rb)
    sim.set_strip(autotune.lookup_strip3(case.nx, case.ny, case.nz))
    orc = O3.Oracle3(case)
    sim.step(5)
    orc.step(5)
    compare(sim.fields(), orc.fields(), 2e-5, "fracture 256x128x30 step 5")
    sim.step(295)
    orc.step(295)
    compare(sim.fields(), orc.fields(), 5e-5, "fracture 256x128x30 step 300",
            ["phi", "T", "fl", "fs", "rhoH", "C", "chi", "rho"])


@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 1, 3), (1, 4, 1), (3, 2, 7)])
def test_degenerate_lattices(lbf_mod, O3, shape):
    nx, ny, nz = shape
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    mat = W.Material()
    z = np.zeros((nz, ny, nx))
    case = W3.Case3(f"deg_{nx}x{ny}x{nz}", nx, ny, nz, (nx % 2 == 1, False, True),
                    [1, 0, 1, 0, 0, 0], [-1.0, 0.0, -0.5, 0.0, 0.0, 0.0], z.copy(), z.copy(),
                    rng.uniform(-1, 1, (nz, ny, nx)), rng.uniform(-0.5, 0.5, (nz, ny, nx)), mat)
    sim = lbf_mod.Sim3(case)
    orc = O3.Oracle3(case)
    sim.step(3)
    orc.step(3)
    compare(sim.fields(), orc.fields(), 2e-5, case.name, ["phi", "T", "fs", "rhoH", "C", "chi"])



def test_long_run_sessile(lbf_mod, O3):
    """1000 steps of the freezing sessile drop (30 x 26 x 22): phi, T and the
    liquid fraction within 1e-4 of the oracle, the bar of the 2D long run."""
    case = cases()["sessile3_30x26x22"]
    sim, orc = lbf_mod.Sim3(case), O3.Oracle3(case)
    sim.step(1000)
    orc.step(1000)
    g, o = sim.fields(), orc.fields()
    assert o["fs"].max() > 0.5
    compare(g, o, 1e-4, "sessile3 1000 steps", ["phi", "T", "fl", "fs"])


def test_strip_order_does_not_change_the_fields(lbf_mod):
    """Every node's arithmetic is the same in any strip order: the fields
    after 12 steps are bit-identical for strips of 1, 3, 16 rows and the
    x-fastest order (ragged last strips included)."""
    case = cases()["sessile3_30x26x22"]
    out = []
    for rows in (1, 3, 16, case.ny):
        sim = lbf_mod.Sim3(case)
        sim.set_strip(rows)
        sim.step(12)
        out.append(sim.fields())
    for f in out[1:]:
        for k in ("phi", "T", "fs", "ux", "uz", "p", "rhoH"):
            assert np.array_equal(out[0][k], f[k]), k


def test_save_and_load_continue_bit_identically(lbf_mod):
    """A checkpoint taken after 15 steps and loaded into a fresh simulation
    of the same case continues bit for bit; a state of another lattice is
    refused."""
    import torch
    a = lbf_mod.Sim3(cases()["boxed_21x19x17"])
    a.step(15)
    buf = torch.empty(a.state_bytes(), dtype=torch.uint8, device="cuda")
    a.save_state(buf)
    a.step(10)
    b = lbf_mod.Sim3(cases()["boxed_21x19x17"])
    b.step(3)
    b.load_state(buf)
    assert b.reduce()["step"] == 15
    b.step(10)
    Fa, Fb = a.fields(), b.fields()
    for k in FIELDS3:
        assert np.array_equal(Fa[k], Fb[k]), k
    other = lbf_mod.Sim3(cases()["sphere_24"])
    with pytest.raises(lbf_mod.LbfError, match="needed"):
        other.load_state(buf)
    big = torch.empty(other.state_bytes(), dtype=torch.uint8, device="cuda")
    other.save_state(big)
    with pytest.raises(lbf_mod.LbfError):
        b.load_state(big)
