"""Pins of the oracle's smoothed aggregation (Section 2.5 readings).

* SplitMix64 against its published output sequence;
* MIS-2: independent in the distance-2 graph and every non-root has a
  higher-priority root within distance 2 -- together these determine the
  greedy set uniquely;
* aggregates: a partition with one root each, connected, root neighbours in
  the root's aggregate, the remaining nodes attached through a neighbour;
* SPAI-0 is the minimiser of ||I - M A||_F over diagonal M (perturbation);
* the smoothed prolongation equals (I - M A) T densely, on the union pattern.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path, connected_components

import synth
from oracle import assembly, sa, ptransfer, hierarchy

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_vector():
    vals = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    assert [sa.splitmix64(1234567, i) for i in range(5)] == vals


def _p1_operator(n, perturb=0.1, seed=4, lam=1.0, bc="dirichlet"):
    m = synth.hex_mesh(n, 1, perturb=perturb, seed=seed)
    A, cons = assembly.assemble(m.coords, m.l2g, 1, lam, bc=bc)
    free = np.nonzero(~cons)[0]
    return A[free][:, free].tocsr()


def _distances(A):
    G = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    G.setdiag(0)
    G.eliminate_zeros()
    return shortest_path(G, unweighted=True), G


@pytest.mark.parametrize("n,seed", [(6, 0), (7, 99)])
def test_mis2_characterisation(n, seed):
    A = _p1_operator(n)
    roots = sa.mis2(A, seed)
    dist, _ = _distances(A)
    prio = sa.priorities(A.shape[0], seed)
    R = np.array(roots)
    sub = dist[np.ix_(R, R)]
    np.fill_diagonal(sub, np.inf)
    assert sub.min() >= 3
    rootset = set(roots)
    for v in range(A.shape[0]):
        if v in rootset:
            continue
        near = R[dist[v, R] <= 2]
        assert any(prio[r] > prio[v] for r in near)


@pytest.mark.parametrize("n,seed", [(6, 0), (8, 5)])
def test_aggregate_invariants(n, seed):
    A = _p1_operator(n)
    agg, roots = sa.aggregate(A, seed)
    dist, G = _distances(A)
    assert agg.min() == 0 and agg.max() == roots.size - 1
    for a, r in enumerate(roots):
        members = np.nonzero(agg == a)[0]
        assert agg[r] == a
        assert np.sum(np.isin(members, roots)) == 1
        sub = G[members][:, members]
        assert connected_components(sub, directed=False)[0] == 1
        nb = G.indices[G.indptr[r]:G.indptr[r + 1]]
        assert np.all(agg[nb] == a)
    # the roots are numbered in increasing node order
    assert np.all(np.diff(roots) > 0)
    # a node at distance 2 from every root joins the highest-priority root at
    # distance 2 (each such root is reached through one of its neighbours)
    prio = sa.priorities(A.shape[0], seed)
    for v in range(A.shape[0]):
        d = dist[v, roots]
        if d.min() == 2:
            best = max((r for r in roots[d == 2]), key=lambda r: prio[r])
            assert agg[v] == agg[best]


def test_spai0_is_frobenius_minimiser():
    A = _p1_operator(3, lam=3.0)
    m = sa.spai0(A)
    D = A.toarray()
    I = np.eye(D.shape[0])
    base = np.linalg.norm(I - np.diag(m) @ D)
    rng = np.random.default_rng(0)
    for i in rng.choice(D.shape[0], 5, replace=False):
        for eps in (1e-3, -1e-3):
            mm = m.copy()
            mm[i] += eps
            assert np.linalg.norm(I - np.diag(mm) @ D) > base


def test_smoothed_prolongation_dense():
    A = _p1_operator(5, lam=2.0)
    agg, roots = sa.aggregate(A, 3)
    P, m, T = sa.smoothed_prolongation(A, agg, roots.size)
    dense = (np.eye(A.shape[0]) - np.diag(m) @ A.toarray()) @ T.toarray()
    np.testing.assert_allclose(P.toarray(), dense, atol=1e-15)
    pat = (galerkin_pattern(A) @ (T.toarray() > 0).astype(int) + (T.toarray() > 0)) > 0
    assert np.array_equal(_struct(P), pat)


def galerkin_pattern(A):
    return sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape).toarray().astype(int)


def _struct(M):
    return sp.csr_matrix((np.ones(M.nnz), M.indices, M.indptr), shape=M.shape).toarray() > 0


def test_hierarchy_sizes_p2_12cube():
    # a p = 2 problem on 12^3 elements reaches h-levels (p1 level > 2000 rows)
    m = synth.hex_mesh(12, 2, perturb=0.1, seed=2)
    H = hierarchy.build(m.coords, m.l2g, 2, 10.0,
                        hierarchy.Options(coarse_max=500))
    kinds = [lv.kind for lv in H.levels]
    assert kinds[:2] == ["p", "p"] and kinds[-1] == "coarsest"
    assert H.levels[1].A.shape[0] == 11 ** 3
    assert H.levels[-1].A.shape[0] <= 500
    for lv, nxt in zip(H.levels[:-1], H.levels[1:]):
        assert lv.P.shape == (lv.A.shape[0], nxt.A.shape[0])


def _anisotropic_2d(nx, ny, eps):
    """5-point operator on an nx x ny grid, node iy * nx + ix: coupling -1
    along x, -eps along y, diagonal 2 + 2 eps (Dirichlet closure)."""
    n = nx * ny
    rows, cols, vals = [], [], []
    for iy in range(ny):
        for ix in range(nx):
            i = iy * nx + ix
            rows.append(i); cols.append(i); vals.append(2.0 + 2.0 * eps)
            for dx, dy, w in ((1, 0, -1.0), (-1, 0, -1.0), (0, 1, -eps), (0, -1, -eps)):
                jx, jy = ix + dx, iy + dy
                if 0 <= jx < nx and 0 <= jy < ny:
                    rows.append(i); cols.append(jy * nx + jx); vals.append(w)
    return assembly.csr_from_sorted_or_not(np.array(rows), np.array(cols), np.array(vals), n, n)


def test_strength_threshold_semicoarsens_anisotropy():
    """With a strength threshold the aggregates follow the strong direction
    (the textbook behaviour of smoothed aggregation on an anisotropic
    operator): every aggregate lies in one grid row and is a run of
    consecutive nodes; with theta = 0 the weak couplings count and
    aggregates cross rows."""
    nx, ny = 17, 9
    A = _anisotropic_2d(nx, ny, 0.01)
    agg, roots = sa.aggregate(A, 5, theta=0.25)
    iy = np.arange(nx * ny) // nx
    ix = np.arange(nx * ny) % nx
    for a in range(roots.size):
        mem = np.nonzero(agg == a)[0]
        assert np.unique(iy[mem]).size == 1
        xs = np.sort(ix[mem])
        assert (np.diff(xs) == 1).all() and 1 <= xs.size <= 5
    agg0, roots0 = sa.aggregate(A, 5, theta=0.0)
    assert any(np.unique(iy[agg0 == a]).size > 1 for a in range(roots0.size))
    assert roots.size > roots0.size


def test_strength_graph_is_symmetric_union():
    """An edge that passes the threshold in one direction only is kept in
    both; a node with no strong neighbour is a root of its own aggregate."""
    A = sp.csr_matrix(np.array([[4.0, -1.0, 0.0, -0.1],
                                [-0.9, 4.0, -1.0, 0.0],
                                [0.0, -1.0, 4.0, 0.0],
                                [-0.1, 0.0, 0.0, 4.0]]))
    # threshold theta * 4 = 0.96: (0,1) passes as -1.0, its mirror -0.9 fails
    nb = sa.neighbours(A, theta=0.24)
    assert nb == [[1], [0, 2], [1], []]
    agg, roots = sa.aggregate(A, 0, theta=0.24)
    assert 3 in set(roots.tolist()) and (agg == agg[3]).sum() == 1
