"""The GIAMG V-cycle (oracle, test infrastructure only).

Algorithm 1 and the paragraph after it (Section 2.1): on the coarsest level
solve directly; otherwise pre-smooth, form the residual r_f = b_f - A_f x_f
explicitly, restrict r_c = R r_f, recurse on the error equation
A_c e_c = r_c, prolong e_f = P e_c, correct x_f = x_f + e_f and post-smooth.
Pre-smoothing starts from the zero vector; post-smoothing continues from the
corrected iterate.
"""
import numpy as np
import scipy.linalg as sla

from . import smoothers


def coarse_solve(level, f):
    if f.size == 0:
        return f.copy()
    y = sla.solve_triangular(level.chol, f, lower=True)
    return sla.solve_triangular(level.chol.T, y, lower=False)


def smooth(H, level, f, x0):
    o = H.opts
    if o.smoother == "chebyshev":
        return smoothers.chebyshev(level.A, level.dinv, f, x0, o.degree,
                                   o.cheb_lo * level.lam_hat,
                                   o.cheb_hi * level.lam_hat)
    if o.smoother == "jacobi":
        return smoothers.jacobi(level.A, level.dinv, f, x0, o.degree, o.omega)
    raise ValueError(o.smoother)


def vcycle(H, f, l=0):
    """One V-cycle on level l applied to right-hand side f (zero initial
    guess); returns the approximation to A_l^-1 f."""
    level = H.levels[l]
    if l == len(H.levels) - 1:
        return coarse_solve(level, f)
    x = smooth(H, level, f, None)
    r = f - level.A @ x
    fc = level.R @ r
    ec = vcycle(H, fc, l + 1)
    x = x + level.P @ ec
    x = smooth(H, level, f, x)
    return x
