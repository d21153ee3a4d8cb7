"""GPU parity of the porous pre-processing (needs a device): the
Cahn-Hilliard smoothing against the FP64 oracle on 2D and 3D images (walls,
wrap, ragged and degenerate sizes, 0 to 500 Euler steps), the host and device
entry paths and caller/library workspaces bit for bit, the full-size images
of the measurement after two steps, and the whole preparation (smoothing,
then phase separation of the pore mixture by the coupled step) against the
oracle, with the saturation conserved."""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2510_18688_amd import lbf, porous
    lbf.load()
    return porous


@pytest.fixture(scope="module")
def CH():
    from oracle import ch_oracle
    return ch_oracle


IMAGES = {
    "2d_walls_53x37": ((37, 53), (False, False)),
    "2d_wrap_x_64x40": ((40, 64), (True, False)),
    "2d_wrap_both_31x29": ((29, 31), (True, True)),
    "3d_mixed_23x20x17": ((17, 20, 23), (False, True, False)),
    "3d_walls_16x9x12": ((12, 9, 16), (False, False, False)),
}


@pytest.mark.parametrize("name", list(IMAGES))
@pytest.mark.parametrize("iters, tol", [(0, 0.0), (1, 1e-6), (40, 5e-6), (500, 2e-5)])
def test_ch_smoothing_matches_oracle(P, CH, name, iters, tol):
    shape, per = IMAGES[name]
    img = W.sandpack_image(shape, seed=len(name) + iters, r_median=3.5, periodic=per)
    g = P.ch_smooth(img, per, iters)
    o = CH.smooth(img, per, iters)
    err = float(np.abs(g.astype(np.float64) - o).max())
    print(name, iters, f"{err:.1e}", flush=True)
    assert err <= tol, (name, iters, err)


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (6, 1), (1, 1, 4), (3, 1, 1), (2, 2, 2)])
def test_ch_degenerate_images(P, CH, shape):
    rng = np.random.default_rng(sum(shape))
    img = (rng.random(shape) < 0.5).astype(np.uint8)
    for per in [(False,) * 3, (True,) * 3]:
        g = P.ch_smooth(img, per[:len(shape)], 30)
        o = CH.smooth(img, per[:len(shape)], 30)
        assert np.abs(g - o).max() <= 5e-6, (shape, per)


def test_ch_device_path_and_workspace(P):
    import torch
    img = W.sandpack_image((48, 40, 32), seed=3, r_median=4.0)
    per = (False, True, True)
    a = P.ch_smooth(img, per, 50)
    t = torch.as_tensor(img, device="cuda")
    b = P.ch_smooth(t, per, 50)
    assert torch.equal(torch.as_tensor(a, device="cuda"), b)
    from paper_2510_18688_amd import lbf
    L = lbf.load()
    p = P.ch_params(img.shape, per)
    ws = torch.empty(L.lbf_ch_workspace_bytes(p.nx, p.ny, p.nz), dtype=torch.uint8, device="cuda")
    c = P.ch_smooth(t, per, 50, workspace=ws)
    assert torch.equal(b, c)


@pytest.mark.parametrize("shape, per", [((2048, 4096), (False, False)),
                                        ((256, 256, 256), (False, True, True))])
def test_ch_full_size_two_steps(P, CH, shape, per):
    img = W.sandpack_image(shape, seed=12, periodic=per)
    g = P.ch_smooth(img, per, 2)
    o = CH.smooth(img, per, 2)
    err = float(np.abs(g.astype(np.float64) - o).max())
    print(shape, f"{err:.1e}", flush=True)
    assert err <= 1e-6


def test_preparation_with_gravity_matches_oracle(P, CH):
    """The separation stage under gravity (the body force of the paper's
    porous stage) against the oracle, 800 steps."""
    from oracle import oracle as O
    img = W.sandpack_image((48, 64), seed=22, r_median=5.0)
    sim, case = P.prepare(img, S_w=0.4, theta_deg=45.0, ch_iterations=300,
                          separation_steps=800, gravity=(0.0, -2e-5))
    assert case.mat.g_y == -2e-5
    phi0 = CH.smooth(img, (False, False, True), 300)
    orc = O.Oracle(W.unsaturated_medium(phi0, S_w=0.4, theta_deg=45.0, gravity=(0.0, -2e-5)))
    orc.step(800)
    g, o = sim.fields(), orc.fields()
    for k in ("phi", "T", "C"):
        assert float(np.abs(g[k] - o[k]).max()) <= 2e-5, k


def test_preparation_matches_oracle(P, CH):
    """Smoothing, then 1500 steps of phase separation of the uniform pore
    mixture (S_w = 0.32, theta = 60 degrees) against the oracle run on the
    oracle's own phi0.  The total phase field (so S_w) changes only by the
    phase-field source phi div u with the flow's own divergence (R54): the
    GPU's S_w matches the oracle's, and both stay at 0.32 to 2e-5."""
    from oracle import oracle as O
    img = W.sandpack_image((64, 96), seed=21, r_median=5.0)
    sim, case = P.prepare(img, S_w=0.32, theta_deg=60.0, ch_iterations=500,
                          separation_steps=1500)
    phi0 = CH.smooth(img, (False, False, True), 500)
    orc = O.Oracle(W.unsaturated_medium(phi0, S_w=0.32, theta_deg=60.0))
    orc.step(1500)
    g, o = sim.fields(), orc.fields()
    for k in ("phi", "T", "C", "rho"):
        err = float(np.abs(g[k] - o[k]).max())
        print(k, f"{err:.1e}", flush=True)
        assert err <= 2e-5, (k, err)
    for k in ("ux", "uy", "p"):
        scale = float(np.abs(o[k]).max())
        assert float(np.abs(g[k] - o[k]).max()) <= 1e-3 * scale + 1e-9, k
    r = sim.reduce()
    Vp = float(np.sum(1.0 - case.phi0))
    S_w = 0.5 * (1.0 + r["sum_g"] / Vp)
    S_wo = 0.5 * (1.0 + orc.reduce()["sum_g"] / float(np.sum(1.0 - phi0)))
    assert abs(S_w - S_wo) < 2e-6, (S_w, S_wo)
    assert abs(S_w - 0.32) < 2e-5, S_w
    assert r["sum_fs"] == 0.0
