"""Column and row profiles of an oracle state, and the freezing observables
built from them (plain numpy, FP64).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).  Definitions
(the readings behind the figure-level quantities of the paper):
  * ice thickness of a column: the sum over its nodes of the ice fraction
    f_s; phase-change-material (PCM) thickness: the sum of chi;
  * top of a column: the highest height at which chi (or f_s) crosses 1/2
    from above, by linear interpolation between the two nodes around the
    crossing (the top row itself when it is at or above 1/2, -1 when no node
    is);
  * row sums of f_s and chi, and the outermost 1/2-crossings of each in a
    row: the leftmost rise and the rightmost fall, interpolated the same way
    (the edge node itself when it is at or above 1/2, -1 when no node is);
  * freezing-front height of a one-dimensional column (Sec. 4.2, the
    three-phase Stefan problem): the ice thickness; final solid height h_f
    (Table 1): the ice thickness after complete freezing;
  * maximum drop height (Sec. 4.4): the highest column top of chi;
  * three-phase contact line (Fig. 6): the highest row above the substrate in
    which the ice reaches the outer edge of the phase-change material on both
    sides (ice edges within half a node of the PCM edges); R_tr is half the
    PCM width of that row, H_tr its height above the substrate;
  * solid fraction (Fig. 13): total ice over total PCM.
"""

from __future__ import annotations

from typing import Dict

import numpy as np


def column_top(v: np.ndarray) -> np.ndarray:
    """Highest 1/2-crossing of each column of v [ny, nx] (see above)."""
    ny, nx = v.shape
    out = np.full(nx, -1.0)
    for x in range(nx):
        col = v[:, x]
        for y in range(ny - 1, -1, -1):
            if col[y] >= 0.5:
                if y == ny - 1:
                    out[x] = float(y)
                else:
                    out[x] = y + (col[y] - 0.5) / (col[y] - col[y + 1])
                break
    return out


def row_edges(v: np.ndarray):
    """Leftmost rising and rightmost falling 1/2-crossing of each row."""
    ny, nx = v.shape
    left = np.full(ny, -1.0)
    right = np.full(ny, -1.0)
    for y in range(ny):
        r = v[y]
        for x in range(nx):
            if r[x] >= 0.5:
                left[y] = 0.0 if x == 0 else x - (r[x] - 0.5) / (r[x] - r[x - 1])
                break
        for x in range(nx - 1, -1, -1):
            if r[x] >= 0.5:
                right[y] = float(x) if x == nx - 1 else x + (r[x] - 0.5) / (r[x] - r[x + 1])
                break
    return left, right


def profiles(F: Dict[str, np.ndarray]) -> Dict[str, Dict[str, np.ndarray]]:
    """Profiles of a fields dict (keys "fs" and "chi", arrays [ny, nx])."""
    fs = np.asarray(F["fs"], dtype=np.float64)
    chi = np.asarray(F["chi"], dtype=np.float64)
    pl, pr = row_edges(chi)
    il, ir = row_edges(fs)
    return {"col": {"ice": fs.sum(0), "pcm": chi.sum(0), "pcm_top": column_top(chi),
                    "ice_top": column_top(fs)},
            "row": {"ice": fs.sum(1), "pcm": chi.sum(1), "pcm_left": pl, "pcm_right": pr,
                    "ice_left": il, "ice_right": ir}}


def solid_fraction(p) -> float:
    return float(p["col"]["ice"].sum() / p["col"]["pcm"].sum())


def contact_line(p, base_row: int):
    """(R_tr, H_tr) of a single drop on a substrate whose first fluid row is
    base_row; None while no row's ice reaches the drop's edge."""
    r = p["row"]
    best = None
    for y in range(base_row, r["pcm"].size):
        if min(r["pcm_left"][y], r["ice_left"][y]) < 0:
            continue
        if r["ice_left"][y] <= r["pcm_left"][y] + 0.5 and r["ice_right"][y] >= r["pcm_right"][y] - 0.5:
            best = y
    if best is None:
        return None
    return 0.5 * float(r["pcm_right"][best] - r["pcm_left"][best]), float(best - base_row)
