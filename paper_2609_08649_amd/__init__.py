"""lensfield: MI355X (gfx950) HIP implementation of the lens-equation hot path of
parametric strong-lens modeling (arXiv 2609.08649).

`paper_2609_08649_amd.lensfield` is the ctypes binding of the C ABI in
include/lensfield.h; `paper_2609_08649_amd.workloads` holds the seeded synthetic
workload generators.  The binding (and torch) is imported lazily.
"""
__all__ = ["lensfield", "workloads", "build"]
