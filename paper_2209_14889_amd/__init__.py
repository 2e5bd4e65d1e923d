"""MI355X (gfx950) implementation of the coupled viscoelastic immersed-boundary lattice Boltzmann
step of arXiv 2209.14889: a HIP library behind the C ABI in include/lb.h, with a thin ctypes
binding (``paper_2209_14889_amd.lb``), seeded workloads (``.workload``) and the MLP surrogate of
the restoring-force series (``.surrogate``).

Importing the package loads nothing; the HIP library is opened on first use.
"""
__all__ = ["lb", "workload"]
