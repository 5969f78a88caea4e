"""MI355X-native coupled immersed-boundary lattice-Boltzmann timestep.

The compute path is the HIP library ``libibl.so`` (hand-written gfx950
kernels behind the C-ABI declared in ``include/ibl.h``); ``ibl`` is its thin
Python binding.  ``workloads`` builds the seeded synthetic inputs.  Importing
this package loads nothing; the library is loaded on first use.
"""
__all__ = ["ibl", "workloads"]
