"""GIAMG hierarchy setup (oracle, test infrastructure only).

Section 2 (Algorithms 1-7 and the h-coarsening subsection): starting from the
assembled fine operator, p-coarsen level by level down to order 1 (Section
2.2 and 2.4), then build smoothed-aggregation levels (Section 2.5) while the
level is larger than ``coarse_max`` rows; every coarse operator is the
Galerkin product R A P with R = P^T, computed at setup (Section 2.1).  The
coarsest level is solved directly (the paper uses SuperLU; here a dense
Cholesky factorisation, which gives the same solution up to rounding).

The modal basis (appendix) uses injection P (Algorithm 7 as printed); the
order-1 level is the same in both bases (vertex modes are the Q1 nodes), so
the smoothed-aggregation levels below it do not depend on the basis.

Readings: p-coarsening always continues to order 1 (Table 1: p = 8 on eight
elements gives four levels); h-levels stop when the level has at most
``coarse_max`` rows, when the hierarchy holds ``max_levels`` levels, or when
aggregation no longer reduces the size; a level that would be empty is not
created.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from . import assembly, ptransfer, sa, galerkin, smoothers


@dataclass
class Level:
    A: sp.csr_matrix
    kind: str                       # "p", "h" or "coarsest"
    order: int                      # polynomial order (1 for h-levels)
    dinv: np.ndarray = None
    lam_hat: float = 0.0
    P: Optional[sp.csr_matrix] = None   # to the next coarser level
    R: Optional[sp.csr_matrix] = None
    l2g: Optional[np.ndarray] = None    # element map (p-levels)
    collect: Optional[np.ndarray] = None
    agg: Optional[np.ndarray] = None
    spai: Optional[np.ndarray] = None
    chol: Optional[np.ndarray] = None   # coarsest: lower Cholesky factor


@dataclass
class Options:
    smoother: str = "chebyshev"     # or "jacobi"
    degree: int = 2                 # Chebyshev degree / Jacobi sweeps
    omega: float = 2.0 / 3.0
    coarse_max: int = 2000
    max_levels: int = 10
    bc: str = "dirichlet"           # or "pin"
    pin: int = 0
    seed: int = 0                   # aggregation priority seed
    theta: float = 0.0              # strength threshold of the aggregation graph
    power_iters: int = 20
    cheb_lo: float = 0.1
    cheb_hi: float = 1.1
    basis: str = "nodal"            # or "modal" (appendix basis, injection P)
    schedule: Optional[List[int]] = None   # coarse orders after p (default q = p / spf(p))
    keep_boundary: bool = False     # coarse p-levels keep the constrained nodes (see build)


@dataclass
class Hierarchy:
    levels: List[Level] = field(default_factory=list)
    opts: Options = None
    constrained: np.ndarray = None


def build(coords, l2g, p, lam, opts: Options = None) -> Hierarchy:
    opts = opts or Options()
    n = coords.shape[0]
    A, cons = assembly.assemble(coords, l2g, p, lam, bc=opts.bc, pin=opts.pin, basis=opts.basis)
    H = Hierarchy(opts=opts, constrained=cons)
    # The paper says boundary nodes need care but not how (Section 2.2.2).
    # Default reading: coarse levels hold the free nodes only (P has empty
    # rows for constrained fine nodes).  keep_boundary: every node passes to
    # the coarse levels, the fine identity rows entering the Galerkin product
    # as P_B^T P_B; on 2^3 elements at p = 8 this gives Table 1's coarsest
    # level of 27 rows and 343 nonzeros.
    free = np.ones(n, dtype=bool) if opts.keep_boundary else ~cons
    cur_l2g = l2g
    orders = ptransfer.p_schedule(p, opts.schedule)
    level = Level(A=A, kind="p", order=p, l2g=l2g)
    H.levels.append(level)
    for q in orders[1:]:
        if len(H.levels) >= opts.max_levels:
            break
        collect, l2g_nx, P = ptransfer.p_level(cur_l2g, level.order, q,
                                               level.A.shape[0], free, opts.basis)
        if collect.size == 0:
            break
        R = galerkin.transpose(P)
        Ac = galerkin.rap(R, level.A, P)
        level.P, level.R, level.collect = P, R, collect
        level = Level(A=Ac, kind="p", order=q, l2g=l2g_nx)
        H.levels.append(level)
        cur_l2g = l2g_nx
        free = np.ones(Ac.shape[0], dtype=bool)
    while (level.order == 1 and level.A.shape[0] > opts.coarse_max
           and len(H.levels) < opts.max_levels):
        agg, roots = sa.aggregate(level.A, opts.seed, opts.theta)
        n_agg = roots.size
        if n_agg >= level.A.shape[0] or n_agg == 0:
            break
        P, m, _ = sa.smoothed_prolongation(level.A, agg, n_agg)
        R = galerkin.transpose(P)
        Ac = galerkin.rap(R, level.A, P)
        level.P, level.R, level.agg, level.spai = P, R, agg, m
        level = Level(A=Ac, kind="h", order=1)
        H.levels.append(level)
    # smoother data on every non-coarsest level; Cholesky on the coarsest
    for lv in H.levels[:-1]:
        lv.dinv = smoothers.diag_inverse(lv.A)
        lv.lam_hat = smoothers.lambda_max_estimate(lv.A, lv.dinv, opts.power_iters)
    last = H.levels[-1]
    last.kind = "coarsest"
    if last.A.shape[0]:
        last.chol = np.linalg.cholesky(last.A.toarray())
    return H
