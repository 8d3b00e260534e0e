"""MI355X-native solver for the all-at-once KKT system of parabolic optimal
control, preconditioned by the epsilon-circulant RBD preconditioner.

The compute path is libpcop.so (HIP kernels for gfx950 behind the C ABI of
include/pcop.h); :mod:`paper_2410_22686_amd.pcop` is its Python binding.
Importing this package does not touch the GPU.
"""
from .pcop import (KKTSolve, NotConverged, PcopError, Solver, SolveInfo, halfgrid_samples,  # noqa: F401
                   kkt_solve, load_library)

__all__ = ["Solver", "SolveInfo", "KKTSolve", "kkt_solve", "PcopError", "NotConverged", "load_library",
           "halfgrid_samples"]
