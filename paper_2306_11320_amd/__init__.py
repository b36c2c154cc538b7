"""MI355X-native (gfx950, HIP) implementation of the per-time-step update of the
three coupled D2Q9 lattice Boltzmann equations of Wang, He & Wang,
"Phase-field-based lattice Boltzmann model for simulating thermocapillary
flows" (arXiv:2306.11320).

The compute path is the C-ABI shared library built from ``csrc/`` (see
``include/lbm.h``); ``lbm`` is its ctypes binding.  Importing this package does
not load the library; ``from paper_2306_11320_amd import lbm`` does.
"""
__all__ = ["lbm", "workloads"]
