"""MI355X-native coupled lattice Boltzmann freezing step (arXiv 2510.18688).

Submodules:
  lbf        ctypes binding of liblbf.so (the HIP step, read-out, reductions)
  workloads  seeded synthetic inputs (no method arithmetic)
  build      hipcc build of liblbf.so
The binding is imported lazily so that input generation works without a GPU.
"""

__all__ = ["lbf", "workloads", "build"]
