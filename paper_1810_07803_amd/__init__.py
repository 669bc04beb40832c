"""MI355X (gfx950) half-range lattice Boltzmann solver for rarefied planar Couette flow.

The solver itself is libhrlb.so (HIP kernels + C ABI, include/hrlb.h); ``hrlb`` is its ctypes
binding.  ``build`` compiles the library in-tree.
"""
from . import hrlb  # noqa: F401
