"""Pins of explicit p-schedules (the paper's by-one schedule, Section 3.4's
schedule study) in the nodal basis, where a coarse step q need not divide p:
the order-q GLL points are then not fine points, a fine lattice node only
numbers each coarse node, and P interpolates.

* P reproduces every Q_q polynomial exactly at the fine nodes (uniform
  mesh, affine elements: a global polynomial of degree <= q per variable is
  in both spaces);
* nested spaces: R A P equals the order-q operator assembled directly with
  the same quadrature (Galerkin identity), for 5 -> 4 and 6 -> 4;
* the by-one hierarchy solves like any other.
"""
import numpy as np
import pytest

import synth
from oracle import assembly, basis, hierarchy, krylov, ptransfer


def _element_points(m, p, e, n):
    """Physical GLL points (order p) of element e of an n^3 uniform mesh."""
    xg, _ = basis.gll_points(p)
    ez, ey, ex = e % n, (e // n) % n, e // (n * n)
    h = 1.0 / n
    t = (xg + 1.0) / 2.0
    return (ex + t) * h, (ey + t) * h, (ez + t) * h


@pytest.mark.parametrize("p,q", [(5, 4), (6, 4), (5, 3), (4, 3), (3, 2)])
def test_interpolation_reproduces_coarse_polynomials(p, q):
    n = 2
    m = synth.hex_mesh(n, p)
    free = np.ones(m.n_nodes, dtype=bool)
    collect, l2g_nx, P = ptransfer.p_level(m.l2g, p, q, m.n_nodes, free)
    rng = np.random.default_rng(p * 10 + q)
    cx, cy, cz = rng.standard_normal((3, q + 1))

    def u(x, y, z):
        return (np.polynomial.polynomial.polyval(x, cx) * np.polynomial.polynomial.polyval(y, cy)
                * np.polynomial.polynomial.polyval(z, cz))

    uc = np.full(collect.size, np.nan)
    uf = np.full(m.n_nodes, np.nan)
    for e in range(m.n_elem):
        X, Y, Z = _element_points(m, q, e, n)
        for a in range(q + 1):
            for b in range(q + 1):
                for c in range(q + 1):
                    uc[l2g_nx[e, assembly.local_index(q, a, b, c)]] = u(X[a], Y[b], Z[c])
        X, Y, Z = _element_points(m, p, e, n)
        for i in range(p + 1):
            for j in range(p + 1):
                for k in range(p + 1):
                    uf[m.l2g[e, assembly.local_index(p, i, j, k)]] = u(X[i], Y[j], Z[k])
    assert not np.isnan(uc).any() and not np.isnan(uf).any()
    assert np.max(np.abs(P @ uc - uf)) <= 1e-12 * np.max(np.abs(uf))


@pytest.mark.parametrize("p,q", [(5, 4), (6, 4)])
def test_non_divisor_galerkin_is_direct_assembly(p, q):
    n = 2
    mp = synth.hex_mesh(n, p, perturb=0.1, seed=5)
    mq = synth.hex_mesh(n, q, perturb=0.1, seed=5)
    Ap, cons = assembly.assemble(mp.coords, mp.l2g, p, 3.0)
    Aq, _ = assembly.assemble(mq.coords, mq.l2g, q, 3.0, nq=p + 2, bc="none")
    collect, l2g_nx, P = ptransfer.p_level(mp.l2g, p, q, mp.n_nodes, ~cons)
    qid = np.full(collect.size, -1, dtype=np.int64)
    for e in range(mp.n_elem):
        for a in range((q + 1) ** 3):
            c = l2g_nx[e, a]
            if c >= 0:
                qid[c] = mq.l2g[e, a]
    assert np.all(qid >= 0)
    Ac = (P.T @ Ap @ P).tocsr()
    ref = Aq[qid][:, qid]
    assert np.max(np.abs((Ac - ref).toarray())) <= 1e-12 * abs(ref).max()


def test_schedule_validation_and_by_one_solve():
    with pytest.raises(ValueError):
        ptransfer.p_schedule(5, [5, 1])
    with pytest.raises(ValueError):
        ptransfer.p_schedule(5, [3, 4, 1])
    assert ptransfer.p_schedule(5, [4, 3, 2, 1]) == [5, 4, 3, 2, 1]
    assert ptransfer.p_schedule(6) == [6, 3, 1]
    m = synth.hex_mesh(3, 5, perturb=0.1, seed=2)
    H = hierarchy.build(m.coords, m.l2g, 5, 2.0, hierarchy.Options(schedule=[4, 3, 2, 1], coarse_max=50))
    assert [lv.order for lv in H.levels] == [5, 4, 3, 2, 1]
    b = synth.normal_rhs(m.n_nodes, 1)
    r = krylov.giamg_pcg(H, b, tol=1e-10)
    import scipy.sparse.linalg as spla
    x = spla.spsolve(H.levels[0].A.tocsc(), b)
    assert r.converged and np.linalg.norm(r.x - x) <= 1e-8 * np.linalg.norm(x)
