"""Launch-shape and plane-stride autotuner of the step kernel.

For a lattice size it times every candidate launch shape (threads per block
along x, rows per block along y) with HIP events on the simulation's stream
and persists the fastest in tiles.json next to this file, keyed by "NXxNY".
`tune_pad` does the same for the padding between the workspace's planes
(lbf_params.plane_pad) of the plane-major layout (and of the 3D lattice),
which decides how the 34 planes that one step streams spread over the HBM
channels; `tune_layout` picks the 2D state layout (rows per block,
lbf_params.row_block) together with its pad.  Their effect depends on the
exact size, so `lookup_pad` and `lookup_layout` answer for measured sizes
only.
"""

from __future__ import annotations

import json
import os
from typing import Iterable, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
DB = os.path.join(HERE, "tiles.json")

CANDIDATES: Tuple[Tuple[int, int], ...] = tuple(
    (tx, ty) for tx in (64, 128, 256, 512) for ty in (1, 2, 4, 8, 16, 32, 64, 128))


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
    sizes = [k for k in db if k.count("x") == 1 and "tile" in db[k]]
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


PAD_CANDIDATES: Tuple[int, ...] = (0, 64, 128, 192, 320, 576, 1088, 2112, 4160, 4224, 6208,
                                   8256, 12352, 16448)


def _key(*size: int) -> str:
    return "x".join(str(int(v)) for v in size)


def lookup_pad(*size: int) -> int:
    """Tuned plane padding of a lattice size (nx, ny) or (nx, ny, nz), 0 if
    that size was not measured."""
    v = _load().get(_key(*size))
    return int(v.get("pad", 0)) if v else 0


def tune_pad(case, tile: Optional[Sequence[int]] = None, steps: int = 100, repeats: int = 3,
             candidates: Iterable[int] = PAD_CANDIDATES, save: bool = True
             ) -> Tuple[int, dict]:
    """Time the step of `case` (2D, with launch shape `tile`, or 3D) with
    each plane padding (a fresh simulation each, median of `repeats` runs of
    `steps` steps) and keep the best."""
    import statistics
    from . import lbf
    three = hasattr(case, "nz")
    times = {}
    for pad in candidates:
        sim = (lbf.Sim3(case, plane_pad=pad, row_block=0) if three
               else lbf.Sim(case, tile=tile, plane_pad=pad, row_block=0))
        sim.step(10)
        sim.set_timing(True)
        runs = []
        for _ in range(repeats):
            sim.step(steps)
            runs.append(sim.last_step_ms() if three else sim.last_step_kernel_ms())
        times[str(pad)] = statistics.median(runs)
        sim.close()
        del sim
    best = int(min(times, key=times.get))
    if save:
        db = _load()
        key = _key(case.nx, case.ny, case.nz) if three else _key(case.nx, case.ny)
        entry = db.get(key, {} if three else {"tile": list(tile)})
        entry["pad"], entry["pad_ms"] = best, times[str(best)]
        entry["pad_all"] = times
        db[key] = entry
        with open(DB, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
    return best, times


# (rows per block, plane pad) of the 2D state layout; row_block 0 is plane-major
LAYOUT_CANDIDATES: Tuple[Tuple[int, int], ...] = tuple(
    (rb, pad) for rb in (0, 2, 4, 8) for pad in (0, 64, 128, 576, 2112, 4160))


def lookup_layout(nx: int, ny: int) -> Tuple[int, int]:
    """Tuned (row_block, plane_pad) of a 2D lattice size; for a size not
    measured, rows of every plane in blocks of one row up to 512 columns
    (the batch of 64 lattices 64 .. 512 wide: 0.321 ms per step against 0.351
    in 4-row blocks) and of four rows above (2048^2), without pad."""
    v = _load().get(_key(nx, ny))
    if v and "layout" in v:
        rb, pad = v["layout"]
        return int(rb), int(pad)
    return (1 if nx <= 512 else 4), 0


def lookup_layout3(nx: int, ny: int, nz: int) -> Tuple[int, int]:
    """Tuned (row_block, plane_pad) of a D3Q19 lattice size; (32, 0) if that
    size was not measured."""
    v = _load().get(_key(nx, ny, nz))
    if v and "layout" in v:
        rb, pad = v["layout"]
        return int(rb), int(pad)
    return 32, 0


def lookup_strip3(nx: int, ny: int, nz: int) -> int:
    """Tuned rows per strip of the D3Q19 step pass's node order
    (lbf3_set_strip); 16 if that size was not measured."""
    v = _load().get(_key(nx, ny, nz))
    return int(v.get("strip", 16)) if v else 16


def tune_layout(case, tile: Optional[Sequence[int]] = None, steps: int = 100, repeats: int = 3,
                candidates: Iterable[Sequence[int]] = LAYOUT_CANDIDATES, save: bool = True
                ) -> Tuple[Tuple[int, int], dict]:
    """Time the 2D step of `case` with launch shape `tile` in each state
    layout (a fresh simulation each, median of `repeats` runs of `steps`
    steps) and keep the best."""
    import statistics
    from . import lbf
    times = {}
    for rb, pad in candidates:
        sim = lbf.Sim(case, tile=tile, plane_pad=pad, row_block=rb)
        sim.step(10)
        sim.set_timing(True)
        runs = []
        for _ in range(repeats):
            sim.step(steps)
            runs.append(sim.last_step_kernel_ms())
        times[f"{rb}/{pad}"] = statistics.median(runs)
        sim.close()
        del sim
    best = min(times, key=times.get)
    layout = tuple(int(v) for v in best.split("/"))
    if save:
        db = _load()
        key = _key(case.nx, case.ny)
        entry = db.get(key, {"tile": list(tile)})
        entry["layout"], entry["layout_ms"] = list(layout), times[best]
        entry["layout_all"] = times
        db[key] = entry
        with open(DB, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
    return layout, times


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
