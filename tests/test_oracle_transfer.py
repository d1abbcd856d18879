"""Pins of the oracle's p-transfers (Algorithms 2-4, 7) and Galerkin RAP.

* 1-D interpolation values against closed-form quadratic Lagrange values;
* P reproduces coarse polynomials at fine nodes on uniform meshes;
* the Galerkin identity: for nested spaces P^T A P is the order-q operator
  assembled directly with the fine quadrature, values and structure;
* brute-force dense R A P and boolean structure on tiny meshes.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import assembly, ptransfer, galerkin

S37 = math.sqrt(3 / 7)
CLOSED_GLL = {1: [-1.0, 1.0], 2: [-1.0, 0.0, 1.0],
              3: [-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0],
              4: [-1.0, -S37, 0.0, S37, 1.0]}


def test_schedule():
    assert ptransfer.p_schedule(8) == [8, 4, 2, 1]
    assert ptransfer.p_schedule(6) == [6, 3, 1]
    assert ptransfer.p_schedule(5) == [5, 1]
    assert ptransfer.p_schedule(4) == [4, 2, 1]
    assert ptransfer.p_schedule(1) == [1]


def test_interp_4_to_2_closed_form():
    I1 = ptransfer.interp_1d(4, 2)
    l0 = lambda x: x * (x - 1) / 2
    l1 = lambda x: 1 - x * x
    l2 = lambda x: x * (x + 1) / 2
    expect = np.array([[l(x) for l in (l0, l1, l2)] for x in CLOSED_GLL[4]])
    expect[np.abs(expect) < 1e-12] = 0
    np.testing.assert_allclose(I1, expect, atol=1e-15)
    assert I1[1, 1] == pytest.approx(4 / 7)
    np.testing.assert_allclose(ptransfer.interp_1d(2, 1), [[1, 0], [.5, .5], [0, 1]], atol=1e-16)


def _lattice_positions(n, p):
    g = np.array(CLOSED_GLL[p])
    lat = []
    for e in range(n):
        lat.extend(((e + (g[:-1] + 1) / 2) / n).tolist())
    lat.append(1.0)
    return np.array(lat)


@pytest.mark.parametrize("p,q", [(2, 1), (4, 2), (3, 1)])
def test_polynomial_reproduction(p, q):
    n = 3
    m = synth.hex_mesh(n, p)
    _, cons = assembly.assemble(m.coords, m.l2g, p, 0.0, bc="pin", pin=0)
    collect, l2g_nx, P = ptransfer.p_level(m.l2g, p, q, m.n_nodes, ~cons)
    lf = _lattice_positions(n, p)
    X, Y, Z = np.meshgrid(lf, lf, lf, indexing="ij")
    xf, yf, zf = X.ravel(), Y.ravel(), Z.ravel()
    # coarse node positions: the coarse lattice of order q
    lc = _lattice_positions(n, q)
    Lq = n * q + 1
    # coarse ids are ranks of kept fine ids; recover the coarse lattice index
    s = p // q
    Lp = n * p + 1
    ix, iy, iz = collect // (Lp * Lp), (collect // Lp) % Lp, collect % Lp
    xc, yc, zc = lc[ix // s], lc[iy // s], lc[iz // s]
    assert Lq == n * q + 1
    for f in (lambda x, y, z: x + 2 * y - 3 * z,
              lambda x, y, z: x * y + z * (x ** q) + y ** q * z):
        uc = f(xc, yc, zc)
        uf = P @ uc
        ref = f(xf, yf, zf)
        ref[cons] = 0.0
        np.testing.assert_allclose(uf, ref, atol=1e-13)


@pytest.mark.parametrize("n,p,q,bc", [(3, 2, 1, "dirichlet"), (3, 4, 2, "dirichlet"),
                                      (2, 4, 2, "pin"), (2, 6, 3, "dirichlet"),
                                      (2, 3, 1, "pin")])
def test_galerkin_identity(n, p, q, bc):
    m = synth.hex_mesh(n, p, perturb=0.15, seed=11)
    lam = 2.5 if bc == "dirichlet" else 0.0
    A, cons = assembly.assemble(m.coords, m.l2g, p, lam, bc=bc)
    collect, l2g_nx, P = ptransfer.p_level(m.l2g, p, q, m.n_nodes, ~cons)
    Ac = galerkin.rap(galerkin.transpose(P), A, P)
    # direct order-q assembly on the same geometry with the fine quadrature
    mq = synth.hex_mesh(n, q, perturb=0.15, seed=11)
    Aq, consq = assembly.assemble(mq.coords, mq.l2g, q, lam, bc=bc,
                                  pin=0, nq=p + 2)
    # map order-q lattice ids to coarse ids through the kept fine nodes
    s = p // q
    Lp, Lq = n * p + 1, n * q + 1
    ix, iy, iz = collect // (Lp * Lp), (collect // Lp) % Lp, collect % Lp
    qid = ((ix // s) * Lq + iy // s) * Lq + iz // s
    ref = Aq[qid][:, qid]
    assert np.array_equal(np.sort(qid), np.nonzero(~consq)[0])
    D = (Ac - ref).toarray()
    assert np.max(np.abs(D)) <= 1e-12 * np.max(np.abs(ref.toarray()))
    # structure: the order-q pattern on free nodes (the product adds no entries)
    Sref = (galerkin.pattern_of(ref) != 0).astype(int)
    Sac = (galerkin.pattern_of(Ac) != 0).astype(int)
    assert (Sref != Sac).nnz == 0
    # l2g_next maps every element's kept nodes consistently
    kept = m.l2g[:, ptransfer.extract_next_dof(p, q)]
    ok = l2g_nx >= 0
    assert np.array_equal(collect[l2g_nx[ok]], kept[ok])
    assert np.all(cons[kept[~ok]])


@pytest.mark.parametrize("n,p,q", [(2, 2, 1), (2, 4, 2)])
def test_rap_bruteforce_dense(n, p, q):
    m = synth.hex_mesh(n, p, perturb=0.2, seed=5)
    A, cons = assembly.assemble(m.coords, m.l2g, p, 1.0)
    _, _, P = ptransfer.p_level(m.l2g, p, q, m.n_nodes, ~cons)
    R = galerkin.transpose(P)
    Ac = galerkin.rap(R, A, P)
    dense = P.toarray().T @ A.toarray() @ P.toarray()
    assert np.max(np.abs(Ac.toarray() - dense)) <= 1e-13 * np.abs(dense).max()
    boolean = ((np.abs(R.toarray()) > 0).astype(np.int64)
               @ galerkin.pattern_of(A).toarray().astype(np.int64)
               @ (np.abs(P.toarray()) > 0).astype(np.int64)) > 0
    assert np.array_equal(galerkin.pattern_of(Ac).toarray() > 0, boolean)
    assert np.max(np.abs((Ac - Ac.T).toarray())) <= 1e-14 * np.abs(dense).max()
    # duplicate-free CSR with ascending columns
    for M in (P, R, Ac):
        for i in range(M.shape[0]):
            cols = M.indices[M.indptr[i]:M.indptr[i + 1]]
            assert np.all(np.diff(cols) > 0)
