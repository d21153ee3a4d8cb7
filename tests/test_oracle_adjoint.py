"""Pins of the FP64 gradient oracle (no GPU).

The PyTorch oracle recomputes the C oracle's discrete map with whole-lattice
tensor operations; autograd then gives the exact gradient of a loss of the
final ice fraction with respect to the per-node wettability cos(theta) and
the wall temperatures, through the initialisation and every step.  Pinned
by (1) agreement of its forward map with the C oracle to round-off and
(2) FP64 central finite differences of the C oracle along random directions.
"""

import numpy as np
import pytest
import torch

from paper_2510_18688_amd import workloads as W


def small_freezing_case():
    return W.small_freezing_case()


def test_torch_oracle_matches_c_oracle(oracle_mod):
    from oracle import torch_oracle as TO
    for case in (W.sessile_drop(nx=40, ny=30, radius=10.0),
                 W.curved_substrate(n=64, R_s=14.0, R_0=10.0),
                 W.porous_medium(nx=90, ny=60, seed=11, rmin=6.0, rmax=9.0, porosity=0.8),
                 small_freezing_case()):
        M, _, _, _ = TO.run(case, 40)
        o = oracle_mod.Oracle(case)
        o.step(40)
        F = o.fields()
        for k in ("phi", "T", "fs", "rhoH", "C", "chi", "rho"):
            assert np.abs(M[k].detach().numpy() - F[k]).max() < 1e-12, (case.name, k)


def loss_and_grads(case, steps, target):
    from oracle import torch_oracle as TO
    M, cth, wallT, _ = TO.run(case, steps, requires_grad=True)
    J = 0.5 * ((M["fs"] - torch.from_numpy(target)) ** 2).sum()
    J.backward()
    return float(J.detach()), cth.grad.numpy().copy(), wallT.grad.numpy().copy()


def oracle_loss(oracle_mod, case, steps, target):
    o = oracle_mod.Oracle(case)
    o.step(steps)
    fs = o.fields()["fs"]
    return 0.5 * float(((fs - target) ** 2).sum())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_autograd_gradient_matches_central_differences(oracle_mod, seed):
    case = small_freezing_case()
    steps = 60
    rng = np.random.default_rng(10 + seed)
    target = 0.3 * rng.uniform(0, 1, (case.ny, case.nx))
    J, g_cth, g_wall = loss_and_grads(case, steps, target)
    assert np.abs(g_cth).max() > 0 and np.abs(g_wall[0, :case.nx]).max() > 0
    # random direction over the per-column contact angles and the bottom-wall profile
    d_th = rng.normal(size=case.nx)
    d_tw = rng.normal(size=case.nx)
    d_th /= np.linalg.norm(d_th)
    d_tw /= np.linalg.norm(d_tw)
    analytic = float((g_cth * d_th[None, :]).sum() + (g_wall[0, :case.nx] * d_tw).sum())
    eps = 1e-6
    vals = []
    for sgn in (1, -1):
        c = small_freezing_case()
        c.cos_theta = c.cos_theta + sgn * eps * d_th[None, :]
        c.wall_T = {W.BOTTOM: c.wall_T[W.BOTTOM] + sgn * eps * d_tw}
        vals.append(oracle_loss(oracle_mod, c, steps, target))
    fd = (vals[0] - vals[1]) / (2 * eps)
    assert abs(fd - analytic) <= 1e-5 * abs(fd) + 1e-9, (fd, analytic)


def test_autograd_gradient_brute_force_every_parameter(oracle_mod):
    """Every parameter of a 16 x 16, 50-step problem (cos theta at all 256
    nodes and the 16 bottom-wall temperatures) by FP64 central differences
    of the C oracle."""
    from oracle import torch_oracle as TO
    case = W.small_freezing_case(nx=16, ny=16, h_s=3.0, radius=5.0, T_wall=-2.0, seed=4)
    steps = 50
    rng = np.random.default_rng(20)
    target = 0.3 * rng.uniform(0, 1, (case.ny, case.nx))
    M, cth, wallT, _ = TO.run(case, steps, requires_grad=True)
    J = 0.5 * ((M["fs"] - torch.from_numpy(target)) ** 2).sum()
    J.backward()
    ad = np.concatenate([cth.grad.numpy().ravel(), wallT.grad.numpy()[0, :case.nx]])
    assert np.count_nonzero(ad) > 100
    eps = 1e-6
    fd = np.zeros_like(ad)
    base_c, base_w = case.cos_theta.copy(), case.wall_T[W.BOTTOM].copy()
    # 544 runs of a 256-node lattice: one thread each (no fork/join per row)
    L = oracle_mod.lib()
    threads0 = L.orc_max_threads()
    L.orc_set_threads(1)
    try:
        _brute_force(oracle_mod, ad, fd, base_c, base_w, steps, target, eps)
    finally:
        L.orc_set_threads(threads0)
    scale = float(np.abs(ad).max())
    assert float(np.abs(fd - ad).max()) <= 1e-6 * scale, (float(np.abs(fd - ad).max()), scale)


def _brute_force(oracle_mod, ad, fd, base_c, base_w, steps, target, eps):
    for k in range(ad.size):
        vals = []
        for sgn in (1.0, -1.0):
            c = W.small_freezing_case(nx=16, ny=16, h_s=3.0, radius=5.0, T_wall=-2.0, seed=4)
            cc, ww = base_c.copy(), base_w.copy()
            if k < cc.size:
                cc.flat[k] += sgn * eps
            else:
                ww[k - cc.size] += sgn * eps
            c.cos_theta, c.wall_T = cc, {W.BOTTOM: ww}
            vals.append(oracle_loss(oracle_mod, c, steps, target))
        fd[k] = (vals[0] - vals[1]) / (2 * eps)


def test_stored_gradient_reference_is_pinned_by_its_differences():
    """tests/golden/c5_gradient.json (256 x 256, 2000 steps): the stored FP64
    autograd gradient against the stored FP64 central differences of the C
    oracle along the same 16 directions, at the smallest step."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c5_gradient.json")))
    g = np.asarray(ref["grad"])
    assert g.size == 512 and abs(ref["J_autograd"] - ref["J0"]) <= 1e-12 * ref["J0"]
    rng = np.random.default_rng(ref["direction_seed"])
    fd = ref["fd"]["1e-06"]
    for k in range(ref["directions"]):
        d = rng.normal(size=g.size)
        d /= np.linalg.norm(d)
        ad = float(g @ d)
        assert abs(ad - fd[k]) <= 1e-5 * abs(ad) + 1e-7 * np.linalg.norm(g), (k, ad, fd[k])
        # the larger steps converge towards it (first-order branch effects)
        assert abs(ref["fd"]["0.0001"][k] - ad) >= abs(fd[k] - ad) or abs(fd[k] - ad) < 1e-7
