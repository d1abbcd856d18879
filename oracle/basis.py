"""1-D nodal and modal bases and quadrature (oracle, test infrastructure only).

The paper's nodal variant builds prolongation by evaluating the lower-order
basis at the higher-order nodes (Introduction; footnote to Algorithm 7).  The
nodal basis used here is the Lagrange basis on the Gauss-Lobatto-Legendre
(GLL) points; the paper does not fix the node set, GLL is the reading.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gll_points(p: int):
    """GLL points and weights of order p (p+1 points on [-1, 1]).

    Points: -1, +1 and the roots of P_p'(x).  Weights: 2 / (p (p+1) P_p(x_i)^2).
    """
    if p < 1:
        raise ValueError("p >= 1")
    coef = np.zeros(p + 1)
    coef[p] = 1.0
    if p == 1:
        x = np.array([-1.0, 1.0])
    else:
        inner = npleg.legroots(npleg.legder(coef))
        x = np.concatenate([[-1.0], np.sort(inner.real), [1.0]])
    Pp = npleg.legval(x, coef)
    w = 2.0 / (p * (p + 1) * Pp * Pp)
    return x, w


def gauss_points(m: int):
    """Gauss-Legendre rule with m points on [-1, 1] (numpy's routine)."""
    x, w = npleg.leggauss(m)
    return x, w


def lagrange_eval(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """L[i, q] = l_i(x_q) for the Lagrange basis on ``nodes`` (product form)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = nodes.size
    L = np.ones((n, x.size))
    for i in range(n):
        for j in range(n):
            if j != i:
                L[i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return L


def lagrange_deriv(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[i, q] = l_i'(x_q): sum over m != i of 1/(x_i - x_m) times the
    product over j not in {i, m} of (x - x_j)/(x_i - x_j)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = nodes.size
    D = np.zeros((n, x.size))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(x.size, 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            D[i] += term
    return D


def modal_eval(p: int, x: np.ndarray) -> np.ndarray:
    """V[n, q] = phi_n(x_q), n = 0..p, for the appendix's 1-D modal basis."""
    from scipy.special import eval_jacobi
    x = np.asarray(x, dtype=np.float64)
    V = np.zeros((p + 1, x.size))
    V[0] = (1.0 - x) / 2.0
    V[1] = (1.0 + x) / 2.0
    for n in range(2, p + 1):
        V[n] = (1.0 - x) / 2.0 * (1.0 + x) / 2.0 * eval_jacobi(n - 2, 1, 1, x)
    return V


def modal_deriv(p: int, x: np.ndarray) -> np.ndarray:
    """D[n, q] = phi_n'(x_q): product rule on the bubble, with
    d/dx P^{1,1}_m = (m + 3)/2 P^{2,2}_{m-1}."""
    from scipy.special import eval_jacobi
    x = np.asarray(x, dtype=np.float64)
    D = np.zeros((p + 1, x.size))
    D[0] = -0.5
    D[1] = 0.5
    for n in range(2, p + 1):
        m = n - 2
        J = eval_jacobi(m, 1, 1, x)
        dJ = (m + 3) / 2.0 * eval_jacobi(m - 1, 2, 2, x) if m >= 1 else np.zeros_like(x)
        D[n] = -x / 2.0 * J + (1.0 - x * x) / 4.0 * dJ
    return D
