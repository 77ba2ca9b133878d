"""MI355X-native Trotterized adiabatic evolution of the toric code in two
transverse fields (the Z2 gauge-Higgs model in its mapped form, arXiv
2108.13410): HIP kernels for gfx950 behind the C ABI of include/z2h.h.

``z2h`` is the ctypes binding (same names as the C entry points);
``workloads`` holds the seeded synthetic workload generators.
"""
from . import z2h  # noqa: F401

__all__ = ["z2h"]
