"""MI355X (gfx950) compact Runge-Kutta Flux Reconstruction step.

The scheme runs in the HIP library libcrkfr.so (C ABI in include/crkfr.h);
``crkfr`` is its ctypes binding and ``workloads`` the seeded input generators.
"""
from . import crkfr, workloads  # noqa: F401
from .crkfr import Batch, Mlp, Solver  # noqa: F401
