"""Outer Krylov loops (oracle, test infrastructure only).

Section 2.1 (end): the V-cycle preconditions conjugate gradients, one
V-cycle per iteration, otherwise standard PCG.  Stopping rule (Section
3.1.1): relative residual below 1e-10; read as ||r_k||_2 / ||b||_2 with the
recursively updated, unpreconditioned residual r_k (the comparison runs in
the commented appendix use the unpreconditioned norm).  The flexible variant
(Polak-Ribiere beta, Golub and Ye 1999; Notay 2000) is the outer loop of the
mixed-precision extension and is checked here in double precision.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    converged: bool
    history: List[float] = field(default_factory=list)
    true_relres: float = 0.0
    status: str = "ok"


def pcg(A, b, precond, tol=1e-10, maxit=500, x0=None, flexible=False):
    """Preconditioned CG; ``precond(r)`` returns z = B r.  With
    ``flexible`` the Polak-Ribiere beta (z_k, r_k - r_{k-1}) / (z_{k-1},
    r_{k-1}) replaces (z_k, r_k) / (z_{k-1}, r_{k-1})."""
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return SolveResult(np.zeros(n), 0, True, [0.0], 0.0)
    r = b - A @ x
    hist = [float(np.linalg.norm(r)) / bnorm]
    if hist[-1] < tol:
        return SolveResult(x, 0, True, hist, hist[-1])
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    status = "maxit"
    k = 0
    for k in range(1, maxit + 1):
        q = A @ p
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            status = "breakdown"
            k -= 1
            break
        alpha = rz / pq
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        hist.append(float(np.linalg.norm(r)) / bnorm)
        if hist[-1] < tol:
            status = "ok"
            break
        z = precond(r)
        if flexible:
            rz_new = float(r @ z)
            beta = float(z @ (r - r_old)) / rz
        else:
            rz_new = float(r @ z)
            beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
    true_rel = float(np.linalg.norm(b - A @ x)) / bnorm
    return SolveResult(x, k, status == "ok", hist, true_rel, status)


def giamg_pcg(H, b, tol=1e-10, maxit=500, x0=None, flexible=False):
    """GIAMG-preconditioned CG on the hierarchy's fine operator."""
    from .cycle import vcycle
    return pcg(H.levels[0].A, b, lambda r: vcycle(H, r), tol, maxit, x0,
               flexible)


def jacobi_pcg(A, b, tol=1e-10, maxit=10000):
    """CG preconditioned by the inverse diagonal of A: the diagonally
    preconditioned CG (DCG) that the paper measures GIAMG against
    (Section 3.2, overall comparison), with the same stopping rule."""
    d = A.diagonal().astype(np.float64)
    return pcg(A, b, lambda r: r / d, tol, maxit)
