"""Freezing observables from the library's column and row profiles
(`Sim.profiles()`, the FP64 reductions of `lbf_profiles`).

  * ice thickness (front height of a one-dimensional column, Sec. 4.2; the
    final solid height h_f of Table 1 once everything has frozen): the mean
    over columns of the column sum of f_s;
  * drop height (Sec. 4.4): the highest column top of the phase-change
    fraction chi above a reference height;
  * three-phase contact line (Fig. 6): the highest row at or above the first
    fluid row in which the ice edges lie within half a node of the edges of
    the phase-change material on both sides; R_tr = half the material's width
    in that row, H_tr = its height above the first fluid row;
  * solid fraction (Fig. 13): total ice over total phase-change material.
"""

from __future__ import annotations

from typing import Optional, Tuple

import numpy as np


def ice_thickness(p) -> float:
    return float(np.mean(p["col"]["ice"]))


def solid_fraction(p) -> float:
    total = float(np.sum(p["col"]["pcm"]))
    return float(np.sum(p["col"]["ice"])) / total if total > 0 else 0.0


def drop_height(p, reference: float = 0.0) -> float:
    return float(np.max(p["col"]["pcm_top"])) - reference


def contact_line(p, first_fluid_row: int) -> Optional[Tuple[float, float]]:
    r = p["row"]
    pl, pr, il, ir = r["pcm_left"], r["pcm_right"], r["ice_left"], r["ice_right"]
    ok = (pl >= 0) & (il >= 0) & (il <= pl + 0.5) & (ir >= pr - 0.5)
    ok[:first_fluid_row] = False
    rows = np.nonzero(ok)[0]
    if rows.size == 0:
        return None
    y = int(rows[-1])
    return 0.5 * float(pr[y] - pl[y]), float(y - first_fluid_row)
