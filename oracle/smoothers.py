"""Level smoothers and their parameters (oracle, test infrastructure only).

Section 2.1: every level uses a Jacobi-accelerated Chebyshev smoother for
pre- and post-smoothing; the number of smoothing "iterations" (Table 1:
three; Section 3.2: two) is read as the polynomial degree k, one
Jacobi-preconditioned Chebyshev step each.  The Chebyshev recurrence is
Saad's Chebyshev acceleration (Iterative Methods for Sparse Linear Systems,
2nd ed., Algorithm 12.1) applied to D^-1 A on an interval [a, b].  Readings:
b = 1.1 lam, a = 0.1 lam, with lam estimated by 20 power iterations on
D^-1 A from the start vector v_i = 2 u(h(i)) - 1, u mapping a 64-bit word to
[0, 1) through its top 53 bits, h the SplitMix64 stream of seed 0.  A
weighted-Jacobi smoother (omega = 2/3) is offered as well.
"""
import numpy as np
import scipy.sparse as sp

from .sa import splitmix64


def diag_inverse(A: sp.csr_matrix) -> np.ndarray:
    return 1.0 / A.diagonal()


def power_start(n: int) -> np.ndarray:
    v = np.empty(n)
    for i in range(n):
        v[i] = 2.0 * ((splitmix64(0, i) >> 11) * 2.0 ** -53) - 1.0
    return v


def lambda_max_estimate(A: sp.csr_matrix, dinv: np.ndarray, iters: int = 20) -> float:
    """Power iteration on D^-1 A: v <- w / ||w||, w = D^-1 A v; returns
    ||w|| / ||v|| of the last step."""
    v = power_start(A.shape[0])
    lam = 0.0
    for _ in range(iters):
        w = dinv * (A @ v)
        lam = np.linalg.norm(w) / np.linalg.norm(v)
        v = w / np.linalg.norm(w)
    return float(lam)


def chebyshev(A, dinv, f, x0, k, lo, hi):
    """Degree-k Chebyshev acceleration of Jacobi for A x = f from x0
    (x0 = None means the zero vector, which saves the first product)."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    if x0 is None:
        x = np.zeros_like(f)
        r = dinv * f
    else:
        x = x0.copy()
        r = dinv * (f - A @ x)
    d = r / theta
    for j in range(k):
        x = x + d
        if j == k - 1:
            break
        r = r - dinv * (A @ d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * r
        rho = rho_new
    return x


def jacobi(A, dinv, f, x0, sweeps, omega):
    """``sweeps`` weighted-Jacobi sweeps x <- x + omega D^-1 (f - A x) from
    x0 (None = zero vector; the first sweep then needs no product)."""
    if x0 is None:
        x = omega * dinv * f
        start = 1
    else:
        x = x0.copy()
        start = 0
    for _ in range(start, sweeps):
        x = x + omega * dinv * (f - A @ x)
    return x
