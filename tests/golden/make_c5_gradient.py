"""Write tests/golden/c5_gradient.json: FP64 reference gradient of the
flat-wall freezing workload (256 x 256, 2000 steps) from the oracle only.

Workload: a drop of radius 77 on a diffuse slab (h_s = 10) over a cold
Dirichlet wall, periodic in x.  Controls u = (theta(x) in radians, T_w(x)),
512 values; base theta = 90 degrees, T_w = -1.  Loss
J(u) = 1/2 sum_x (f_l(u) - f_l*)^2 at the final step, with f_l* the oracle's
final liquid fraction for theta* = 90 + 15 s1(x) degrees and
T_w* = -1 + 0.25 s2(x) (s_k: four random periodic Fourier modes,
numpy default_rng(5)).

Stored: J(u), dJ/du from the FP64 autograd oracle (segment-checkpointed), and
FP64 central differences of the C oracle along 16 random unit directions in
R^512 (default_rng(6)) at delta = 1e-4, 1e-5, 1e-6.

    python tests/golden/make_c5_gradient.py   (about half an hour on 8 cores)
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2510_18688_amd import workloads as W  # noqa: E402

STEPS = 2000
DELTAS = (1e-4, 1e-5, 1e-6)
NDIR = 16


def with_controls(case, theta_rad, Tw):
    case.cos_theta = np.broadcast_to(np.cos(theta_rad)[None, :], (case.ny, case.nx)).copy()
    case.wall_T = {W.BOTTOM: np.asarray(Tw, dtype=np.float64).copy()}
    return case


def final_fl(theta_rad, Tw):
    case, _, _ = W.adjoint_case(steps=STEPS)
    o = O.Oracle(with_controls(case, theta_rad, Tw))
    o.step(STEPS)
    return o.fields()["fl"]


def main(out=os.path.join(HERE, "c5_gradient.json")):
    import torch
    from oracle import torch_oracle as TO
    O.build()
    torch.set_num_threads(os.cpu_count() or 8)
    case, th_t, tw_t = W.adjoint_case(steps=STEPS)
    n = case.nx
    t0 = time.time()
    fl_star = final_fl(np.radians(th_t), tw_t)
    print(f"target done {time.time() - t0:.0f}s", flush=True)
    th0 = np.full(n, np.pi / 2)
    tw0 = np.full(n, -1.0)

    def J_of(u):
        fl = final_fl(u[:n], u[n:])
        return 0.5 * float(((fl - fl_star) ** 2).sum())

    u0 = np.concatenate([th0, tw0])
    J0 = J_of(u0)
    print(f"J0 = {J0!r} {time.time() - t0:.0f}s", flush=True)
    # FP64 autograd gradient
    theta = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    tw = torch.tensor(tw0, dtype=torch.float64, requires_grad=True)
    cth = torch.cos(theta)[None, :].expand(case.ny, n)
    zero = torch.zeros(max(case.nx, case.ny), dtype=torch.float64)
    wallT = torch.stack([tw, zero, zero, zero])
    c0 = with_controls(case, th0, tw0)
    M, _ = TO.run_checkpointed(c0, STEPS, cth, wallT, segment=20)
    fl = 1.0 - M["fs"]
    Jt = 0.5 * ((fl - torch.from_numpy(fl_star)) ** 2).sum()
    Jt.backward()
    g = np.concatenate([theta.grad.numpy(), tw.grad.numpy()])
    print(f"autograd J = {float(Jt.detach())!r} |g| = {np.linalg.norm(g):.6e} "
          f"{time.time() - t0:.0f}s", flush=True)
    rng = np.random.default_rng(6)
    dirs = []
    for _ in range(NDIR):
        d = rng.normal(size=2 * n)
        dirs.append(d / np.linalg.norm(d))
    fd = {f"{d:g}": [] for d in DELTAS}
    for k, d in enumerate(dirs):
        for delta in DELTAS:
            jp = J_of(u0 + delta * d)
            jm = J_of(u0 - delta * d)
            fd[f"{delta:g}"].append((jp - jm) / (2 * delta))
        print(f"direction {k}: adjoint {float(g @ d):.9e} fd "
              + " ".join(f"{fd[f'{x:g}'][-1]:.9e}" for x in DELTAS)
              + f" {time.time() - t0:.0f}s", flush=True)
    rec = {
        "workload": "flat-wall freezing, 256 x 256, drop radius 77 on slab h_s = 10, "
                    "theta = 90 deg, T_w = -1, 2000 steps",
        "steps": STEPS,
        "controls": "u = (theta(x) [rad], T_w(x)), bottom wall, x = 0..255",
        "J0": J0,
        "J_autograd": float(Jt.detach()),
        "grad": g.tolist(),
        "direction_seed": 6,
        "directions": NDIR,
        "fd": fd,
        "generated_by": "tests/golden/make_c5_gradient.py (FP64 oracle only)",
    }
    with open(out, "w") as f:
        json.dump(rec, f, indent=0)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    # optional: python make_c5_gradient.py STEPS OUT (a shorter trial run)
    if len(sys.argv) > 2:
        STEPS = int(sys.argv[1])
        main(sys.argv[2])
    else:
        main()
