#!/usr/bin/env python3
"""Throughput of the coupled LB freezing step on one MI355X.

One step = one coupled update (flow, phase field and enthalpy populations)
of every node of the drop-on-a-cold-cylinder workload, a 2048 x 2048 D2Q9
lattice (cylinder radius 400, drop radius 300, contact angle 60 degrees).
The value is whole-lattice MLUPS (million lattice-node updates per second)
with all state resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic HBM bytes per lattice-node update, the method's own count with
# the phase-field source taken from the model's mass source: 27 distributions
# and 5 lagged fields (f_s, Q = rho C_p T mdot, (phi u)_x, (phi u)_y, p) read
# and written in FP32, and 3 static fields read (phi0, cos theta, lap phi0).
# The roofline is priced at this count.
BYTES_PER_LU = (27 + 5) * 2 * 4 + 3 * 4
# The same count with the source from the flow's own divergence (the default
# reading): the previous step's velocity is needed as well, and (phi u) of
# the previous step is then the product of phi and u, so the lagged fields
# are f_s, Q, phi, p, u_x, u_y.
METHOD_BYTES_PER_LU = (27 + 6) * 2 * 4 + 3 * 4
# What this implementation's step kernel moves by design: those 27
# distributions and 6 lagged fields plus one plane holding the 16-bit high
# parts of the float-float rest populations g_0, h_0 (7 lagged planes) read
# and written, and 2 static planes read (phi0, cos theta; lap phi0 is formed
# from phi0 in the kernel).
IMPL_BYTES_PER_LU = (27 + 7) * 2 * 4 + 2 * 4
HBM_PEAK_GBS = 8000.0
# D3Q19, two kernels per step, with the phase-field source from the flow's
# divergence.  Moments pass: g and h pulled (38 planes), the high parts of
# g_0, h_0, f_s, Q and p of the previous step, phi0 and the previous step's
# velocity (3 planes) read; a 16-byte record (phi, f_s, rho, p) and the
# divergence (4 bytes) written.  Step pass: 57 distributions, the 7 other
# lagged planes, 3 static planes, the record and the divergence read; 57
# distributions and 11 lagged planes (8 and the velocity) written.  The state
# itself (one pass, no records) is 556 bytes per update.
BYTES3_MOMENTS = (38 + 5 + 1 + 3) * 4 + 16 + 4
BYTES3_STEP = (57 + 7 + 3) * 4 + 16 + 4 + (57 + 11) * 4
BYTES3_STATE = (57 + 11) * 2 * 4 + 3 * 4
# Cahn-Hilliard smoothing, per node and Euler step (one fused pass): c read
# once and the new c written once.
BYTES_CH = 4 + 4


def hbm_traffic(kernel_ms, name="step_kernel_curved_substrate_2048x2048"):
    """HBM traffic of a kernel from a committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by the same counters'
    reading of a plain 512 MiB copy); None when the kernel sources changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name + ".hbm.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for p in rec["sources"]:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--tile", type=str, default="", help="TXxTY, e.g. 128x32")
    ap.add_argument("--plane-pad", type=int, default=-1,
                    help="floats of padding between workspace planes (-1: the tuned value)")
    ap.add_argument("--row-block", type=int, default=-1,
                    help="rows per block of the state layout, 0 plane-major (-1: the tuned value)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--batch-steps", type=int, default=320,
                    help="steps of the 64-lattice batched workload (0 skips it)")
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="steps of the 256 x 256 gradient workload (0 skips it)")
    ap.add_argument("--adjoint-hbm-steps", type=int, default=200,
                    help="steps of the gradient workload at 2048 x 2048, where the state "
                         "and the tape live in HBM (0 skips it)")
    ap.add_argument("--d3q19-steps", type=int, default=200,
                    help="steps of the D3Q19 workloads (0 skips them)")
    ap.add_argument("--small-steps", type=int, default=5000,
                    help="steps of the 128 x 96 sessile-drop leg (0: skip)")
    ap.add_argument("--porous-steps", type=int, default=1000,
                    help="steps of the 4096 x 2048 porous-medium leg (0: skip)")
    ap.add_argument("--mdot-steps", type=int, default=1000,
                    help="steps of the headline workload with the mass source as div u (0 skips it)")
    ap.add_argument("--mrt-steps", type=int, default=1000,
                    help="steps of the headline workload with the MRT flow collision (0 skips)")
    ap.add_argument("--ch-iterations", type=int, default=500,
                    help="Euler steps of the Cahn-Hilliard smoothing workloads (0 skips them)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run an elementwise copy of MIB MiB (read + write), the "
                         "reference kernel for scaling HBM byte counters")
    return ap.parse_args()


def cpu_baseline(case, seconds):
    """The FP64 oracle as it stands, on the host cores, on a bounded sample:
    whole-lattice steps of the same workload until `seconds` have passed,
    once with every host thread the oracle's OpenMP runtime offers and once
    on one thread."""
    from oracle import oracle as O
    O.build()
    L = O.lib()
    threads = L.orc_max_threads()

    def timed(budget):
        orc = O.Oracle(case)
        steps = 0
        t0 = time.perf_counter()
        while True:
            orc.step(1)
            steps += 1
            dt = time.perf_counter() - t0
            if dt >= budget or steps >= 1000:
                break
        return steps, dt

    steps, dt = timed(seconds)
    L.orc_set_threads(1)
    try:
        steps1, dt1 = timed(seconds / 2)
    finally:
        L.orc_set_threads(threads)
    return {"value": case.nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} whole-lattice FP64 steps of {case.name} ({dt:.1f} s) on "
                      f"{threads} threads; {steps1} steps ({dt1:.1f} s) on 1 thread",
            "value_1core": case.nodes * steps1 / dt1 / 1e6,
            "host_cpus": os.cpu_count()}


def batched(lbf, W, torch, steps):
    """64 uneven droplet lattices: one persistent launch per step (graph
    replays) against the same lattices stepped one after another with their
    own launches."""
    from paper_2510_18688_amd import autotune
    cases = W.batch_instances(64, seed=4)
    nodes = sum(c.nodes for c in cases)
    sims = [lbf.Sim(c) for c in cases]
    for s, c in zip(sims, cases):
        t = autotune.lookup(c.nx, c.ny)
        if t:
            s.set_tile(*t)
    tile = autotune.lookup_batch(len(cases), nodes) or (128, 32)
    batch = lbf.Batch(sims, tile=tile)
    batch.step(64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    for s in sims:
        s.step(8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.step(steps)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    red = [s.reduce(check_stable=False) for s in sims[:3]]
    return {"workload": "64 droplet lattices, sides log-uniform in [64, 512]",
            "lattices": len(cases), "nodes": nodes, "steps": steps,
            "tile": f"{tile[0]}x{tile[1]}", "work_items": batch.items(),
            "batched_mlups": round(nodes * steps / tb / 1e6, 1),
            "serial_mlups": round(nodes * steps / ts / 1e6, 1),
            "speedup": round(ts / tb, 2),
            "nonfinite": sum(r["nonfinite"] for r in red)}


def adjoint(lbf, W, torch, steps, n=256):
    """Gradient workload: a drop on a slab over a cold wall, 256 x 256 (or
    n x n with the drop scaled, for the HBM-resident form).  The forward time
    of `steps` plain steps against the reverse sweep (segment recomputation
    included) of the same run, for J = 1/2 sum (f_l - f_l*)^2 with respect to
    cos(theta) per node and the wall temperatures."""
    radius = 77.0 * n / 256
    case, th_t, tw_t = W.adjoint_case(n=n, steps=steps, radius=radius)
    from paper_2510_18688_amd import autotune
    tile = autotune.lookup(case.nx, case.ny)
    # the target: final liquid fraction under the target controls (any
    # target gives the same work)
    tcase, _, _ = W.adjoint_case(n=n, steps=steps, radius=radius)
    tcase.cos_theta = np.broadcast_to(np.cos(np.radians(th_t))[None, :], (tcase.ny, tcase.nx)).copy()
    tcase.wall_T = {W.BOTTOM: np.asarray(tw_t, dtype=np.float64)}
    sim = lbf.Sim(tcase, tile=tile, row_block=0)
    sim.step(steps)
    fl_star = torch.as_tensor(sim.field("fl"), device="cuda")
    sim.close()
    # forward: plain steps from the initial state (the tape's plane-major layout)
    sim = lbf.Sim(case, tile=tile, row_block=0)
    sim.step(8)
    sim.init_fields(case.phi, case.T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    sim.init_fields(case.phi, case.T)
    tape = lbf.Tape(sim, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tape.forward()
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    fl = torch.as_tensor(sim.field("fl"), device="cuda")
    J = 0.5 * float(((fl.double() - fl_star.double()) ** 2).sum())
    seed_fs = (-(fl - fl_star)).contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gc, gw = tape.backward(seed_fs=seed_fs)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    seg = tape.segment
    tape.close()
    sim.close()
    torch.cuda.empty_cache()
    return {"workload": f"{case.name}: drop R {radius:g} on slab h_s 10 over a cold wall, "
                        "J = 1/2 sum (f_l - f_l*)^2",
            "nodes": case.nodes, "steps": steps, "segment": seg, "J": J,
            "grad_norm_cos_theta": float(gc.norm()), "grad_norm_wall_T": float(gw.norm()),
            "forward_ms": round(t_fwd * 1e3, 2), "tape_forward_ms": round(t_rec * 1e3, 2),
            "backward_ms": round(t_bwd * 1e3, 2),
            "adjoint_over_forward": round(t_bwd / t_fwd, 3),
            "record_and_adjoint_over_forward": round((t_rec + t_bwd) / t_fwd, 3)}


def d3q19(lbf, torch, steps):
    """The three-dimensional coupled step: freezing in a rough fracture
    (256 x 128 x 30, three trapped bubbles, cold inlet face) and a drop in a
    periodic 256^3 box."""
    from paper_2510_18688_amd import autotune, workloads3 as W3
    out = {}
    for label, case in (("fracture_256x128x30", W3.fracture()),
                        ("sphere_drop_256x256x256", W3.sphere_drop(256, 64.0))):
        rb, pad = autotune.lookup_layout3(case.nx, case.ny, case.nz)
        sim = lbf.Sim3(case, plane_pad=pad, row_block=rb)
        strip = autotune.lookup_strip3(case.nx, case.ny, case.nz)
        sim.set_strip(strip)
        sim.step(max(steps // 10, 5))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sim.set_timing(True)
        sim.step(steps)
        ms = sim.last_step_ms()
        sim.set_timing(False)
        red = sim.reduce()
        sim.close()
        del sim
        torch.cuda.empty_cache()
        n = case.nodes
        gbs = (BYTES3_MOMENTS + BYTES3_STEP) * n / (ms * 1e-3) / 1e9
        out[label] = {
            "nodes": n, "steps": steps, "plane_pad": pad, "row_block": rb, "strip": strip,
            "mlups": round(n * steps / wall / 1e6, 1),
            "ms_per_step": round(wall / steps * 1e3, 5),
            "kernel_ms_per_step": round(ms, 5),
            "bytes_per_lu": BYTES3_MOMENTS + BYTES3_STEP,
            "achieved_gbs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "state_bytes_frac": round(BYTES3_STATE * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "nonfinite": red["nonfinite"], "umax": red["umax"],
        }
        rec = hbm_traffic(ms, "d3q19_kernels_" + label) if n == 16777216 else None
        if rec is not None:
            per_lu = sum((k["hbm_bytes_per_launch"] / n) for k in rec["kernels"].values())
            out[label]["traffic_bytes_per_lu"] = round(per_lu, 1)
            out[label]["traffic_gbs"] = round(per_lu * n / (ms * 1e-3) / 1e9, 1)
    return out


def mrt(lbf, W, torch, steps, tile, pad, rb):
    """The headline workload with MRT flow and phase-field collisions (bulk
    rate 1.5, energy-flux rate 1.2, phase-field rate 1.4): the same state and
    bytes per update as BGK."""
    case = W.curved_substrate()
    case.mat.mrt, case.mat.s_b, case.mat.s_q, case.mat.s_g = 1, 1.5, 1.2, 1.4
    sim = lbf.Sim(case, tile=tile, plane_pad=pad, row_block=rb)
    sim.step(50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.set_timing(True)
    sim.step(steps)
    kms = sim.last_step_kernel_ms()
    red = sim.reduce()
    sim.close()
    gbs = BYTES_PER_LU * case.nodes / (kms * 1e-3) / 1e9
    return {"workload": case.name + " with MRT (s_b 1.5, s_q 1.2, s_g 1.4)", "steps": steps,
            "mlups": round(case.nodes * steps / wall / 1e6, 1),
            "kernel_ms": round(kms, 5), "achieved_gbs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "nonfinite": red["nonfinite"]}


def mass_source(lbf, W, torch, steps, tile, pad, rb):
    """The headline workload with the model's mass source as the phase-field
    source's divergence (phi_src_mdot = 1) instead of the previous step's
    velocity divergence: no velocity planes, the lagged (phi u) stored, 272
    bytes per update moved by the kernel; stable over shorter runs only."""
    case = W.curved_substrate()
    case.mat.phi_src_mdot = 1
    sim = lbf.Sim(case, tile=tile, plane_pad=pad, row_block=rb)
    sim.step(50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.set_timing(True)
    sim.step(steps)
    kms = sim.last_step_kernel_ms()
    red = sim.reduce()
    sim.close()
    gbs = BYTES_PER_LU * case.nodes / (kms * 1e-3) / 1e9
    return {"workload": case.name + " with the mass source as div u (phi_src_mdot 1)",
            "steps": steps, "mlups": round(case.nodes * steps / wall / 1e6, 1),
            "kernel_ms": round(kms, 5), "achieved_gbs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "impl_bytes_per_lu": 272,
            "impl_frac": round(272 * case.nodes / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "nonfinite": red["nonfinite"]}


def small(lbf, W, torch, steps):
    """The 128 x 96 sessile drop of the parity runs (5000 steps in the
    paper's set-up): its 3.3 MB of state stay in the caches, so its rate is
    bound by latency, not HBM; reported as MLUPS and time per step."""
    from paper_2510_18688_amd import autotune
    case = W.sessile_drop()
    tile = autotune.lookup(case.nx, case.ny)
    sim = lbf.Sim(case, tile=tile)
    sim.step(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    red = sim.reduce()
    sim.close()
    return {"workload": case.name, "nodes": case.nodes, "steps": steps,
            "tile": f"{tile[0]}x{tile[1]}", "mlups": round(case.nodes * steps / wall / 1e6, 1),
            "us_per_step": round(wall / steps * 1e6, 2), "nonfinite": red["nonfinite"]}


def porous(lbf, W, torch, steps):
    """The complex-geometry workload: 4096 x 2048 porous medium of random
    circular grains (radii 20-60, porosity 0.6), walls on all sides, left
    half liquid, cold left wall, contact angle 45 degrees, mass source on;
    tuned tile and plane padding.  Priced at the same 268 algorithmic B per update as the
    headline workload."""
    from paper_2510_18688_amd import autotune
    case = W.porous_medium()
    tile = autotune.lookup(case.nx, case.ny)
    rb, pad = autotune.lookup_layout(case.nx, case.ny)
    sim = lbf.Sim(case, tile=tile, plane_pad=pad, row_block=rb)
    sim.step(50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.set_timing(True)
    sim.step(steps)
    kms = sim.last_step_kernel_ms()
    red = sim.reduce()
    sim.close()
    gbs = BYTES_PER_LU * case.nodes / (kms * 1e-3) / 1e9
    return {"workload": case.name, "nodes": case.nodes, "steps": steps,
            "tile": f"{tile[0]}x{tile[1]}", "plane_pad": pad, "row_block": rb,
            "mlups": round(case.nodes * steps / wall / 1e6, 1),
            "kernel_ms": round(kms, 5), "achieved_gbs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "nonfinite": red["nonfinite"],
            "solid_fraction": round(red["sum_fs"] / case.nodes, 6)}


def ch_smoothing(torch, iterations):
    """Porous pre-processing: Cahn-Hilliard smoothing of a synthetic sandpack
    image (porosity 0.3585, log-normal grains), 2D 4096 x 2048 with walls and
    3D 256^3 with walls normal to x; image and result resident on the
    device."""
    from paper_2510_18688_amd import lbf, porous, workloads as W
    L = lbf.load()
    porous._declare(L)
    out = {}
    for label, shape, per in (("sandpack_4096x2048", (2048, 4096), (False, False)),
                              ("sandpack_256x256x256", (256, 256, 256), (False, True, True))):
        img = torch.as_tensor(W.sandpack_image(shape, seed=12, periodic=per), device="cuda")
        p = porous.ch_params(shape, per)
        ws = torch.empty(L.lbf_ch_workspace_bytes(p.nx, p.ny, p.nz), dtype=torch.uint8,
                         device="cuda")
        porous.ch_smooth(img, per, 10, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi0 = porous.ch_smooth(img, per, iterations, workspace=ws)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        n = img.numel()
        gbs = BYTES_CH * n * iterations / wall / 1e9
        out[label] = {"nodes": n, "iterations": iterations, "ms": round(wall * 1e3, 3),
                      "us_per_iteration": round(wall / iterations * 1e6, 2),
                      "mlups": round(n * iterations / wall / 1e6, 1),
                      "bytes_per_lu": BYTES_CH, "achieved_gbs": round(gbs, 1),
                      "frac": round(gbs / HBM_PEAK_GBS, 4),
                      "solid_fraction": round(float(phi0.double().mean()), 5)}
        del img, ws, phi0
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the coupled step runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2510_18688_amd import lbf, workloads as W

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.add(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    case = W.curved_substrate()
    from paper_2510_18688_amd import autotune
    rb, pad = autotune.lookup_layout(case.nx, case.ny)
    if args.plane_pad >= 0:
        pad = args.plane_pad
    if args.row_block >= 0:
        rb = args.row_block
    sim = lbf.Sim(case, plane_pad=pad, row_block=rb)
    if args.tile:
        tx, ty = (int(v) for v in args.tile.lower().split("x"))
        sim.set_tile(tx, ty)
    else:
        best = autotune.lookup(case.nx, case.ny)
        if best:
            sim.set_tile(*best)
    tile = sim.tile()
    sim.step(args.warmup)
    torch.cuda.synchronize()

    # timed region: K steps, inputs resident in HBM
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # kernel duration from HIP events on the simulation's stream
    sim.set_timing(True)
    sim.step(args.steps)
    kms = sim.last_step_kernel_ms()
    sim.set_timing(False)
    red = sim.reduce()
    # the same access pattern with no arithmetic: the ceiling the step can reach
    copy_ms, copy_bytes = sim.copy_probe(max(args.steps, 20))

    # observables: column and row profiles of the final state
    from paper_2510_18688_amd import observe
    sim.profiles()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        prof = sim.profiles()
    prof_ms = (time.perf_counter() - t0) / 10 * 1e3

    nodes = case.nodes
    mlups = nodes * args.steps / wall / 1e6
    achieved = BYTES_PER_LU * nodes / (kms * 1e-3) / 1e9
    counters = hbm_traffic(kms)
    traffic = None
    traffic_per_lu = None
    if counters is not None:
        traffic = round(counters["hbm_bytes_per_launch"] / (kms * 1e-3) / 1e9, 1)
        traffic_per_lu = round(counters["hbm_bytes_per_launch"] / nodes, 1)
    out = {
        "metric": "MLUPS of coupled 3-field LB step, % of HBM peak; adjoint/forward time ratio",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": case.name, "nx": case.nx, "ny": case.ny, "nodes": nodes,
                   "tile": f"{tile[0]}x{tile[1]}", "plane_pad": pad, "row_block": rb,
                   "steps_per_run": case.steps},
        "pct_hbm": round(100.0 * mlups * 1e6 * BYTES_PER_LU / (HBM_PEAK_GBS * 1e9), 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "step_kernel",
                     "kernel_ms": round(kms, 5), "bytes_per_lu": BYTES_PER_LU,
                     "impl_bytes_per_lu": IMPL_BYTES_PER_LU,
                     "impl_frac": round(IMPL_BYTES_PER_LU * nodes / (kms * 1e-3) / 1e9
                                        / HBM_PEAK_GBS, 4),
                     "method_bytes_per_lu": METHOD_BYTES_PER_LU,
                     "method_frac": round(METHOD_BYTES_PER_LU * nodes / (kms * 1e-3) / 1e9
                                          / HBM_PEAK_GBS, 4),
                     "traffic_bytes_per_launch": counters and counters["hbm_bytes_per_launch"],
                     "traffic_bytes_per_lu": traffic_per_lu,
                     "traffic_over_algorithmic": counters and round(
                         counters["hbm_bytes_per_launch"] / (BYTES_PER_LU * nodes), 4)},
        "copy_ceiling": {"kernel": "k_copy_probe (the step's planes, tiles and row order; "
                                   "no arithmetic)",
                         "ms": round(copy_ms, 5),
                         "bytes_per_lu": round(copy_bytes / nodes, 1),
                         "gbs": round(copy_bytes / (copy_ms * 1e-3) / 1e9, 1),
                         "frac": round(copy_bytes / (copy_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         # the step's bandwidth (its own bytes) over the copy's
                         "step_bw_over_copy": round(IMPL_BYTES_PER_LU * nodes / kms
                                                    / (copy_bytes / copy_ms), 4)},
        "checks": {"nonfinite": red["nonfinite"], "umax": red["umax"]},
        "observables": {"profiles_ms": round(prof_ms, 3),
                        "solid_fraction": observe.solid_fraction(prof),
                        "drop_top_y": observe.drop_height(prof)},
    }
    del sim
    if args.batch_steps > 0:
        out["batched"] = batched(lbf, W, torch, args.batch_steps)
    if args.adjoint_steps > 0:
        out["adjoint"] = adjoint(lbf, W, torch, args.adjoint_steps)
    if args.adjoint_hbm_steps > 0:
        out["adjoint_hbm"] = adjoint(lbf, W, torch, args.adjoint_hbm_steps, n=2048)
    if args.mrt_steps > 0:
        out["mrt"] = mrt(lbf, W, torch, args.mrt_steps, tile, pad, rb)
    if args.mdot_steps > 0:
        out["mass_source"] = mass_source(lbf, W, torch, args.mdot_steps, tile, pad, rb)
    if args.porous_steps > 0:
        out["porous"] = porous(lbf, W, torch, args.porous_steps)
    if args.small_steps > 0:
        out["small"] = small(lbf, W, torch, args.small_steps)
    if args.d3q19_steps > 0:
        out["d3q19"] = d3q19(lbf, torch, args.d3q19_steps)
    if args.ch_iterations > 0:
        out["ch_smoothing"] = ch_smoothing(torch, args.ch_iterations)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
