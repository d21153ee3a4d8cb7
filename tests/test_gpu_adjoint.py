"""GPU reverse sweep (adjoint with checkpoint recomputation) against the FP64
gradient oracle (needs a device).

The oracle differentiates the FP64 discrete map exactly (PyTorch autograd of
oracle/torch_oracle.py, itself pinned to the C oracle and to central
differences).  The HIP path runs the forward step in FP32 and the reverse
sweep in FP32 with FP64 gradient accumulation.  The bar on every case:
relative L2 error of each gradient (cos theta per node, wall temperatures)
at most 2e-3, cosine similarity at least 0.9999, and on 16 random unit
directions the directional derivative within 1e-3 of the oracle's plus
1e-4 of |grad| (an absolute floor for directions nearly orthogonal to the
gradient).
"""

import numpy as np
import pytest

from paper_2510_18688_amd import workloads as W

pytestmark = pytest.mark.gpu

REL_L2 = 2e-3
COSINE = 0.9999
DIR_REL, DIR_FLOOR = 1e-3, 1e-4


@pytest.fixture(scope="module")
def lbf_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2510_18688_amd import lbf
    lbf.load()
    return lbf


def misfit_loss(target, a_phi=None, a_T=None):
    """J = 1/2 sum (f_s - target)^2 [+ sum a_phi phi + sum a_T T]."""
    def J(F, torch):
        t = torch.as_tensor(target, dtype=torch.float64, device=F["fs"].device)
        out = 0.5 * ((F["fs"] - t) ** 2).sum()
        if a_phi is not None:
            out = out + (torch.as_tensor(a_phi, dtype=torch.float64, device=F["phi"].device)
                         * F["phi"]).sum()
        if a_T is not None:
            out = out + (torch.as_tensor(a_T, dtype=torch.float64, device=F["T"].device)
                         * F["T"]).sum()
        return out
    return J


def oracle_grads(case, steps, loss):
    import torch
    from oracle import torch_oracle as TO
    M, cth, wallT, _ = TO.run(case, steps, requires_grad=True)
    J = loss({"phi": M["phi"], "T": M["T"], "fs": M["fs"]}, torch)
    J.backward()
    g = wallT.grad.numpy() if wallT.grad is not None else np.zeros(tuple(wallT.shape))
    gc = cth.grad.numpy().copy() if cth.grad is not None else np.zeros(tuple(cth.shape))
    nx, ny = case.nx, case.ny
    wall = np.concatenate([g[0, :nx], g[1, :nx], g[2, :ny], g[3, :ny]])
    return float(J.detach()), gc, wall


def gpu_grads(lbf, case, steps, loss, segment=0, tile=None):
    import torch
    cth = torch.tensor(case.cos_theta, dtype=torch.float64, device="cuda", requires_grad=True)
    wall = torch.tensor(lbf.wall_vector(case), dtype=torch.float64, device="cuda",
                        requires_grad=True)
    phi, T, fs = lbf.freeze_fields(cth, wall, case, steps, segment, tile)
    J = loss({"phi": phi.double(), "T": T.double(), "fs": fs.double()}, torch)
    J.backward()
    return float(J.detach()), cth.grad.cpu().numpy(), wall.grad.cpu().numpy()


def check_gradients(label, g_gpu, g_orc, rng):
    report = {}
    for name, a, b in (("cos_theta", g_gpu[0], g_orc[0]), ("wall_T", g_gpu[1], g_orc[1])):
        a = a.ravel()
        b = b.ravel()
        nb = float(np.linalg.norm(b))
        if nb <= 1e-12:
            # no dependence (up to FP64 round-off): the FP32 sweep may leave
            # round-off of its own, nothing more
            assert float(np.abs(a).max()) <= 1e-7, (label, name, float(np.abs(a).max()))
            continue
        rel = float(np.linalg.norm(a - b)) / nb
        cos = float(a @ b) / (float(np.linalg.norm(a)) * nb)
        worst = 0.0
        for _ in range(16):
            d = rng.normal(size=b.size)
            d /= np.linalg.norm(d)
            da, db = float(d @ a), float(d @ b)
            err = abs(da - db)
            worst = max(worst, err / (DIR_REL * abs(db) + DIR_FLOOR * nb))
        report[name] = dict(rel_l2=rel, cosine=cos, dir_ratio=worst)
        assert rel <= REL_L2, (label, name, rel)
        assert cos >= COSINE, (label, name, cos)
        assert worst <= 1.0, (label, name, worst)
    print(label, report, flush=True)
    return report


def run_case(lbf, case, steps, loss, seed=0, segment=0):
    case.mat.phi_src_mdot = 1   # the phase-field source form the reverse sweep supports
    Jg, gc, gw = gpu_grads(lbf, case, steps, loss, segment)
    Jo, oc, ow = oracle_grads(case, steps, loss)
    assert abs(Jg - Jo) <= 1e-3 * abs(Jo) + 1e-6, (case.name, Jg, Jo)
    return check_gradients(case.name, (gc, gw), (oc, ow), np.random.default_rng(100 + seed))


def test_misfit_gradient_small_freezing(lbf_mod):
    case = W.small_freezing_case()
    rng = np.random.default_rng(10)
    target = 0.3 * rng.uniform(0, 1, (case.ny, case.nx))
    run_case(lbf_mod, case, 60, misfit_loss(target))


def test_general_seeds(lbf_mod):
    """Seeds on phi and T as well as f_s."""
    case = W.small_freezing_case(seed=2)
    rng = np.random.default_rng(11)
    target = 0.3 * rng.uniform(0, 1, (case.ny, case.nx))
    a_phi = 0.01 * rng.normal(size=(case.ny, case.nx))
    a_T = 0.01 * rng.normal(size=(case.ny, case.nx))
    run_case(lbf_mod, case, 50, misfit_loss(target, a_phi, a_T), seed=1)


def test_walls_on_all_sides_and_corners(lbf_mod):
    """Porous medium: walls on four sides, Dirichlet left (cold) and right."""
    case = W.porous_medium(nx=48, ny=32, seed=11, rmin=4.0, rmax=6.0, porosity=0.8)
    rng = np.random.default_rng(12)
    target = 0.2 * rng.uniform(0, 1, (case.ny, case.nx))
    run_case(lbf_mod, case, 40, misfit_loss(target, a_T=0.01 * rng.normal(size=(case.ny, case.nx))),
             seed=2)


def test_held_substrate(lbf_mod):
    """Curved substrate with its solid held at the substrate temperature."""
    case = W.curved_substrate(n=48, R_s=10.0, R_0=8.0)
    rng = np.random.default_rng(13)
    target = 0.2 * rng.uniform(0, 1, (case.ny, case.nx))
    run_case(lbf_mod, case, 40, misfit_loss(target, a_T=0.01 * rng.normal(size=(case.ny, case.nx))),
             seed=3)


def test_zero_steps(lbf_mod):
    """No step: only the initial equilibrium and the final moments."""
    case = W.small_freezing_case(seed=3)
    rng = np.random.default_rng(14)
    run_case(lbf_mod, case, 0, misfit_loss(0.1 * rng.uniform(0, 1, (case.ny, case.nx)),
                                           a_phi=0.01 * rng.normal(size=(case.ny, case.nx))),
             seed=4)


def test_checkpoint_interval_does_not_change_the_gradient(lbf_mod):
    """Recomputed segments reproduce the recorded states bit for bit, so every
    checkpoint interval gives the same gradient."""
    case = W.small_freezing_case()
    rng = np.random.default_rng(10)
    loss = misfit_loss(0.3 * rng.uniform(0, 1, (case.ny, case.nx)))
    ref = gpu_grads(lbf_mod, case, 45, loss, segment=45)
    for seg in (1, 7, 0):
        got = gpu_grads(lbf_mod, case, 45, loss, segment=seg)
        assert got[0] == ref[0]
        assert np.array_equal(got[1], ref[1]), seg
        assert np.array_equal(got[2], ref[2]), seg


def test_tape_call_order(lbf_mod):
    lbf = lbf_mod
    case = W.small_freezing_case()
    sim = lbf.Sim(case, row_block=0)
    tape = lbf.Tape(sim, 5, 2)
    assert tape.segment == 2
    with pytest.raises(lbf.LbfError, match="LBF_ESTATE"):
        tape.backward(seed_fs=np.ones((case.ny, case.nx)))
    tape.forward()
    sim.step(1)
    with pytest.raises(lbf.LbfError, match="moved"):
        tape.backward(seed_fs=np.ones((case.ny, case.nx)))
    tape.close()
    sim.close()


def test_gradient_workload_256_against_fp64_reference(lbf_mod):
    """The 256 x 256, 2000-step gradient workload: per-column contact angle
    (radians) and bottom-wall temperature, J = 1/2 sum (f_l - f_l*)^2 with the
    oracle's f_l* of the target controls.  Compared with the stored FP64
    reference (autograd gradient and central differences along 16 random
    unit directions, written by tests/golden/make_c5_gradient.py)."""
    import json
    import os
    import torch
    from oracle import oracle as O
    lbf = lbf_mod
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c5_gradient.json")))
    steps = ref["steps"]
    case, th_t, tw_t = W.adjoint_case(steps=steps)
    n = case.nx
    # target: the oracle's final liquid fraction under the target controls
    O.build()
    tc, _, _ = W.adjoint_case(steps=steps)
    tc.cos_theta = np.broadcast_to(np.cos(np.radians(th_t))[None, :], (n, n)).copy()
    tc.wall_T = {W.BOTTOM: np.asarray(tw_t, dtype=np.float64)}
    o = O.Oracle(tc)
    o.step(steps)
    fl_star = torch.as_tensor(o.fields()["fl"], device="cuda")
    theta = torch.full((n,), np.pi / 2, dtype=torch.float64, device="cuda", requires_grad=True)
    tw = torch.full((n,), -1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    cth = torch.cos(theta)[None, :].expand(n, n).contiguous()
    wall = torch.cat([tw, torch.zeros(n + 2 * n, dtype=torch.float64, device="cuda")])
    phi, T, fs = lbf.freeze_fields(cth, wall, case, steps)
    J = 0.5 * (((1.0 - fs.double()) - fl_star) ** 2).sum()
    J.backward()
    g = np.concatenate([theta.grad.cpu().numpy(), tw.grad.cpu().numpy()])
    gr = np.asarray(ref["grad"])
    Jv = float(J.detach())
    assert abs(Jv - ref["J0"]) <= 1e-3 * ref["J0"], (Jv, ref["J0"])
    cos = float(g @ gr) / (np.linalg.norm(g) * np.linalg.norm(gr))
    rel = float(np.linalg.norm(g - gr) / np.linalg.norm(gr))
    rng = np.random.default_rng(ref["direction_seed"])
    worst = 0.0
    rows = []
    for k in range(ref["directions"]):
        d = rng.normal(size=2 * n)
        d /= np.linalg.norm(d)
        ours, orc = float(g @ d), float(gr @ d)
        fds = [ref["fd"][key][k] for key in ref["fd"]]
        rows.append((ours, orc, fds))
        worst = max(worst, abs(ours - orc) / (1e-3 * abs(orc) + 1e-4 * np.linalg.norm(gr)))
    print("gradient workload", dict(J=Jv, J_ref=ref["J0"], cosine=cos, rel_l2=rel,
                                    dir_ratio=worst), flush=True)
    for r in rows:
        print("  direction", r, flush=True)
    assert cos >= COSINE, cos
    assert worst <= 1.0, worst
