"""MI355X-native (gfx950 HIP) solver for the coupled phase-field + P-u
lattice Boltzmann step of Otomo et al., arXiv 2512.01027.

The compute path is ``libpulbm.so`` (C-ABI, hand-written HIP kernels); the
Python modules here only marshal arguments (``binding``), generate seeded
synthetic inputs (``workloads``) and drive the serving loop (``serving``).
Importing the package does not load the native library.
"""

__all__ = ["binding", "workloads", "serving"]
