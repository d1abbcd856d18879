"""Smoothed-aggregation h-coarsening (oracle, test infrastructure only).

Section 2.5 (h-coarsening): once the order reaches 1, aggregates are formed
from a maximal independent set, the tentative prolongation is piecewise
constant over the aggregates, and it is smoothed with a sparse approximate
inverse (SPAI) smoother (Broeker and Grote, 2002).  The paper defers the
details to its Saena library; the readings taken here:

* graph: the strong off-diagonal couplings of A.  j is a strong neighbour
  of i when |a_ij| >= theta * sqrt(|a_ii a_jj|) (the strength measure of
  Vanek, Mandel and Brezina, 1996); an edge that passes in either direction
  is kept in both, so the graph is symmetric even when the Galerkin
  product's rounding leaves a_ij and a_ji a few ulp apart.  theta = 0 (the
  default) keeps every stored off-diagonal entry, explicit zeros included;
* roots: the greedy maximal independent set of the distance-2 graph (MIS-2)
  taken in decreasing priority order, priority(i) = (h(i), i), where h(i) is
  the (i+1)-th output of SplitMix64 seeded with ``seed`` (Steele, Lea and
  Flood, 2014) and ties go to the larger index;
* aggregates: numbered by increasing root index; every neighbour of a root
  joins it; every remaining node joins, among its already aggregated
  neighbours, the aggregate whose root has the highest priority;
* SPAI-0: m_i = a_ii / sum_j a_ij^2 (the diagonal minimiser of
  ||I - M A||_F);
* P = (I - diag(m) A) T on the symbolic pattern pattern(T) u pattern(A T),
  with no value-based pruning.
"""
import numpy as np
import scipy.sparse as sp

from .galerkin import values_on_pattern, symbolic_product

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, i: int) -> int:
    """(i+1)-th output of SplitMix64 started from state ``seed``."""
    z = (seed + (i + 1) * GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def priorities(n: int, seed: int):
    return [(splitmix64(seed, i), i) for i in range(n)]


def neighbours(A: sp.csr_matrix, theta: float = 0.0):
    """Sorted adjacency lists of the strength graph (see the module notes)."""
    n = A.shape[0]
    diag = np.abs(A.diagonal())
    adj = [set() for _ in range(n)]
    for i in range(n):
        for s in range(A.indptr[i], A.indptr[i + 1]):
            j = int(A.indices[s])
            if j != i and abs(A.data[s]) >= theta * np.sqrt(diag[i] * diag[j]):
                adj[i].add(j)
                adj[j].add(i)
    return [sorted(a) for a in adj]


def mis2(A: sp.csr_matrix, seed: int, theta: float = 0.0):
    """Greedy MIS of the distance-2 graph in decreasing priority order."""
    n = A.shape[0]
    nb = neighbours(A, theta)
    prio = priorities(n, seed)
    order = sorted(range(n), key=lambda i: prio[i], reverse=True)
    blocked = [False] * n
    roots = []
    for v in order:
        if blocked[v]:
            continue
        roots.append(v)
        blocked[v] = True
        for u in nb[v]:
            blocked[u] = True
            for w in nb[u]:
                blocked[w] = True
    return sorted(roots)


def aggregate(A: sp.csr_matrix, seed: int, theta: float = 0.0):
    """Aggregate id per node and the sorted root list (a node with no strong
    neighbour is a root of its own aggregate)."""
    n = A.shape[0]
    nb = neighbours(A, theta)
    prio = priorities(n, seed)
    roots = mis2(A, seed, theta)
    agg = [-1] * n
    root_of = [-1] * n
    for a, r in enumerate(roots):
        agg[r] = a
        root_of[r] = r
    for a, r in enumerate(roots):
        for u in nb[r]:
            agg[u] = a          # unique: roots are at distance >= 3
            root_of[u] = r
    first = list(agg)
    first_root = list(root_of)
    for v in range(n):
        if first[v] >= 0:
            continue
        best = None
        for u in nb[v]:
            if first[u] >= 0:
                r = first_root[u]
                if best is None or prio[r] > prio[best]:
                    best = r
        assert best is not None, "node farther than 2 from every root"
        agg[v] = first[best]
    return np.array(agg, dtype=np.int32), np.array(roots, dtype=np.int64)


def tentative(agg: np.ndarray, n_agg: int) -> sp.csr_matrix:
    n = agg.size
    T = sp.csr_matrix((np.ones(n), agg.astype(np.int32), np.arange(n + 1)),
                      shape=(n, n_agg))
    T.has_sorted_indices = True
    return T


def spai0(A: sp.csr_matrix) -> np.ndarray:
    """m_i = a_ii / sum_j a_ij^2."""
    diag = A.diagonal()
    rowsq = np.asarray(A.multiply(A).sum(axis=1)).ravel()
    return diag / rowsq


def smoothed_prolongation(A: sp.csr_matrix, agg: np.ndarray, n_agg: int):
    """P = (I - diag(m) A) T on pattern(T) u pattern(A T)."""
    T = tentative(agg, n_agg)
    m = spai0(A)
    AT = A @ T
    num = (T - sp.diags(m) @ AT).tocsr()
    pattern = symbolic_product(A, T)
    pattern = ((pattern + T) != 0).astype(np.float64).tocsr()
    pattern.sort_indices()
    return values_on_pattern(pattern, num), m, T
