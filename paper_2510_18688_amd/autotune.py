"""Tile-shape autotuner of the step kernel.

For a lattice size it times every candidate launch shape (threads per block
along x, rows per block along y) with HIP events on the simulation's stream
and persists the fastest in tiles.json next to this file, keyed by "NXxNY".
"""

from __future__ import annotations

import json
import os
from typing import Iterable, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
DB = os.path.join(HERE, "tiles.json")

CANDIDATES: Tuple[Tuple[int, int], ...] = tuple(
    (tx, ty) for tx in (64, 128, 256) for ty in (1, 2, 4, 8, 16, 32, 64, 128))


def _load() -> dict:
    if os.path.exists(DB):
        with open(DB) as f:
            return json.load(f)
    return {}


def lookup(nx: int, ny: int) -> Optional[Tuple[int, int]]:
    """Best known tile for a lattice size: measured, else the nearest size measured."""
    db = _load()
    v = db.get(f"{nx}x{ny}")
    if v:
        return tuple(v["tile"])
    sizes = [k for k in db if not k.startswith("batch")]
    if not sizes:
        return None

    def dist(key):
        a, b = (int(t) for t in key.split("x"))
        return abs(a * b - nx * ny)
    return tuple(db[min(sizes, key=dist)]["tile"])


def tune(sim, steps: int = 20, candidates: Iterable[Sequence[int]] = CANDIDATES,
         save: bool = True) -> Tuple[Tuple[int, int], dict]:
    """Time each candidate on `sim` (its state advances) and keep the best."""
    times = {}
    sim.set_timing(True)
    for tx, ty in candidates:
        sim.set_tile(tx, ty)
        sim.step(2)
        sim.step(steps)
        times[f"{tx}x{ty}"] = sim.last_step_kernel_ms()
    sim.set_timing(False)
    best = min(times, key=times.get)
    tile = tuple(int(v) for v in best.split("x"))
    sim.set_tile(*tile)
    if save:
        db = _load()
        db[f"{sim.nx}x{sim.ny}"] = {"tile": list(tile), "ms": times[best], "all": times}
        with open(DB, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
    return tile, times


BATCH_CANDIDATES: Tuple[Tuple[int, int], ...] = tuple(
    (tx, ty) for tx in (64, 128, 256) for ty in (2, 4, 8, 16, 32, 64))


def lookup_batch(count: int, nodes: int) -> Optional[Tuple[int, int]]:
    """Best known tile of a batched workload of `count` lattices."""
    v = _load().get(f"batch{count}")
    return tuple(v["tile"]) if v else None


def tune_batch(batch, steps: int = 64, candidates: Iterable[Sequence[int]] = BATCH_CANDIDATES,
               save: bool = True) -> Tuple[Tuple[int, int], dict]:
    """Time each tile shape on a batch (its lattices advance) and keep the best."""
    times = {}
    batch.set_timing(True)
    for tx, ty in candidates:
        batch.set_tile(tx, ty)
        batch.step(steps)          # first call builds the work list and the graph
        batch.step(steps)
        times[f"{tx}x{ty}"] = batch.last_step_ms()
    batch.set_timing(False)
    best = min(times, key=times.get)
    tile = tuple(int(v) for v in best.split("x"))
    batch.set_tile(*tile)
    if save:
        db = _load()
        db[f"batch{len(batch.sims)}"] = {"tile": list(tile), "ms": times[best], "all": times}
        with open(DB, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
    return tile, times
