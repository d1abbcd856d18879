"""MI355X-native GIAMG-PCG: GIAMG-preconditioned conjugate gradients for
high-order (GLL-nodal hexahedral) finite-element systems, after Xu, Rasouli,
Kirby, Moxey and Sundar (arXiv 2512.15121).

The solver lives in ``libgiamg.so`` (C ABI declared in include/giamg.h, HIP
kernels for gfx950); ``giamg`` is its ctypes binding.
"""
from .giamg import (Solver, Options, SolveInfo, GiamgError, Session, Server, library,  # noqa: F401
                    read_bandwidth)
