"""Run by tests/test_sanitizers.py in a subprocess with the AddressSanitizer
runtime preloaded: small 2D and 3D oracle runs through the oracles' own
Python wrappers, on sanitizer-instrumented builds of the oracle sources
(paths in LBF_ORC2 and LBF_ORC3)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import oracle as O, oracle3 as O3  # noqa: E402
from paper_2510_18688_amd import workloads as W, workloads3 as W3  # noqa: E402

O.LIB, O3.LIB = os.environ["LBF_ORC2"], os.environ["LBF_ORC3"]
O.build = lambda force=False: O.LIB
O3.build = lambda force=False: O3.LIB

for mdot in (0, 1):
    case = W.sessile_drop(nx=24, ny=18, radius=6.0)
    case.periodic_x = False
    case.thermal_bc = [1, 0, 1, 0]
    case.wall_T = {0: np.full(24, -1.0), 2: np.full(18, -0.5)}
    case.mat.phi_src_mdot = mdot
    o = O.Oracle(case)
    o.step(7)
    f = o.fields()
    assert all(np.isfinite(v).all() for v in f.values())
    st = o.get_state()
    o.set_state(*st)
    o.step(2)
    o.reduce()
case = W.curved_substrate(n=40, R_s=8.0, R_0=6.0)
case.mat.mrt, case.mat.s_b, case.mat.s_q, case.mat.s_g = 1, 1.5, 1.2, 1.4
o = O.Oracle(case)
o.set_isothermal(np.where(np.arange(40 * 40).reshape(40, 40) % 7 == 0, -0.5, np.nan))
o.step(5)
assert np.isfinite(o.fields()["T"]).all()
c3 = W3.sessile_drop3(nx=10, ny=8, nz=7, radius=3.0, h_s=2.0)
o3 = O3.Oracle3(c3)
o3.step(5)
assert all(np.isfinite(v).all() for v in o3.fields().values())
print("oracle runs clean")
