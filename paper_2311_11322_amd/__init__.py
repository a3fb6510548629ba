"""MI355X-native soft-sphere DEM step for rigid bonded-sphere aggregates.

The compute path lives in the HIP shared library built from ``csrc/`` and is
reached through :mod:`paper_2311_11322_amd.dem` (a thin ctypes binding over
the C-ABI declared in ``include/dem.h``).  Importing the package itself loads
nothing, so the seeded input generators in :mod:`.workloads` can be used
without the library.
"""
__all__ = ["workloads", "dem"]
