"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds geometry and random numbers only: structured hexahedral
meshes of the unit cube (optionally with perturbed interior vertices), the
element-to-node map in the tensor ordering the method expects, and random
right-hand sides.  It contains none of the solver's arithmetic (no basis
functions, no quadrature, no assembly), so that the CPU oracle and the HIP
library can both consume it without sharing any of the method's code.
"""
from .mesh import hex_mesh, HexMesh
from .rhs import normal_rhs, pinned_normal_batch, loguniform_lambda

__all__ = ["hex_mesh", "HexMesh", "normal_rhs", "pinned_normal_batch",
           "loguniform_lambda"]
