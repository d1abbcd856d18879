"""Plain FP64 CPU oracle for the GIAMG-preconditioned CG solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP
library; the only common input is the seeded mesh/RHS generator ``synth``.

Every function follows a passage of the paper (Xu, Rasouli, Kirby, Moxey,
Sundar, "A geometrically informed algebraic multigrid preconditioned
iterative approach for solving high-order finite element systems",
arXiv 2512.15121) cited in its docstring, written slowly and plainly in
numpy/scipy double precision.  Where the paper is silent the reading used is
stated in the docstring.

Pins: each function is checked by ``tests/test_oracle_*.py`` against closed
forms, invariants, brute force on tiny inputs or the paper's Table 1.
"""
from . import basis, assembly, ptransfer, sa, galerkin, smoothers, cycle, krylov, hierarchy  # noqa: F401
