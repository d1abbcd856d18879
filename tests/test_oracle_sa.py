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
