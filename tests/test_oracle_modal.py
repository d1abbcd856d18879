"""Pins of the oracle's modal variant (appendix basis; Algorithm 2 as printed;
Algorithm 7 with injected ones).

* the 1-D modes against closed forms in Legendre polynomials, independent
  of the Jacobi evaluation the oracle uses: for n >= 2
  phi_n = (n-1)/(2(2n-1)) (L_{n-2} - L_n) and phi_n' = -(n-1)/2 L_{n-1};
  vertex modes sum to one, bubbles vanish at the ends;
* uniform meshes: the 3-D operator equals the Kronecker sum of 1-D modal
  operators built here by exact polynomial integration, in the modal
  lattice ordering;
* perturbed meshes: the vertex modes carry the constant (volume, K 1 = 0);
* injection: every Galerkin operator is the principal submatrix of the
  finer one on the kept modes, bit for bit, and equals the order-q modal
  operator assembled directly with the same quadrature;
* the Galerkin solution does not depend on the basis: modal and nodal
  solves of the manufactured problem give the same function at every GLL
  node (to solver precision).
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla
from numpy.polynomial import Legendre, Polynomial

import synth
from oracle import assembly, basis, hierarchy, ptransfer
from synth.mesh import modal_positions


def _modal_polys(p):
    """The 1-D modes as numpy polynomials from the Legendre closed forms."""
    x = Polynomial([0.0, 1.0])
    out = [(1 - x) / 2, (1 + x) / 2]
    for n in range(2, p + 1):
        ln2 = Legendre.basis(n - 2).convert(kind=Polynomial)
        ln = Legendre.basis(n).convert(kind=Polynomial)
        out.append((n - 1) / (2.0 * (2 * n - 1)) * (ln2 - ln))
    return out


@pytest.mark.parametrize("p", [1, 2, 3, 5, 6])
def test_modal_basis_closed_forms(p):
    xs = np.linspace(-1, 1, 23)
    V = basis.modal_eval(p, xs)
    D = basis.modal_deriv(p, xs)
    polys = _modal_polys(p)
    for n, poly in enumerate(polys):
        assert np.max(np.abs(V[n] - poly(xs))) < 1e-14
        assert np.max(np.abs(D[n] - poly.deriv()(xs))) < 1e-13
        if n >= 2:
            # derivative of the bubble is -(n-1)/2 L_{n-1}
            ref = -(n - 1) / 2.0 * Legendre.basis(n - 1)(xs)
            assert np.max(np.abs(D[n] - ref)) < 1e-13
            assert abs(V[n][0]) < 1e-15 and abs(V[n][-1]) < 1e-15
    assert np.max(np.abs(V[0] + V[1] - 1.0)) < 1e-15


def _one_d_modal(n, p):
    """1-D modal mass and stiffness on [0, 1] (n elements), exact integration,
    assembled on the lattice positions of the modal ordering."""
    polys = _modal_polys(p)
    h = 1.0 / n
    Me = np.zeros((p + 1, p + 1))
    Ke = np.zeros((p + 1, p + 1))
    for i in range(p + 1):
        for j in range(p + 1):
            pm = (polys[i] * polys[j]).integ()
            pk = (polys[i].deriv() * polys[j].deriv()).integ()
            Me[i, j] = (pm(1) - pm(-1)) * h / 2
            Ke[i, j] = (pk(1) - pk(-1)) * 2 / h
    N = n * p + 1
    M = np.zeros((N, N))
    K = np.zeros((N, N))
    pos = modal_positions(p)
    for e in range(n):
        g = e * p + pos
        M[np.ix_(g, g)] += Me
        K[np.ix_(g, g)] += Ke
    return M, K


@pytest.mark.parametrize("n,p,lam", [(2, 2, 1.0), (2, 3, 0.5), (1, 5, 2.0)])
def test_modal_kronecker_sum_uniform(n, p, lam):
    m = synth.hex_mesh(n, p, basis="modal")
    A, _ = assembly.assemble(m.coords, m.l2g, p, lam, bc="none", basis="modal")
    M1, K1 = _one_d_modal(n, p)
    ref = (np.kron(np.kron(K1, M1), M1) + np.kron(np.kron(M1, K1), M1)
           + np.kron(np.kron(M1, M1), K1) + lam * np.kron(np.kron(M1, M1), M1))
    D = A.toarray()
    assert np.max(np.abs(D - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,p", [(3, 2), (2, 4)])
def test_modal_perturbed_volume_and_nullspace(n, p):
    m = synth.hex_mesh(n, p, perturb=0.15, seed=4, basis="modal")
    Kf, _ = assembly.assemble(m.coords, m.l2g, p, 0.0, bc="none", basis="modal")
    Mf, _ = assembly.assemble(m.coords, m.l2g, p, 1.0, bc="none", basis="modal")
    Mf = Mf - Kf
    # the constant is the sum of the vertex modes (bubbles carry nothing)
    one = np.zeros(m.n_nodes)
    corners = m.l2g[:, assembly.corner_local_indices(p, "modal")].ravel()
    one[corners] = 1.0
    assert abs(one @ (Mf @ one) - 1.0) < 1e-13
    assert np.max(np.abs(Kf @ one)) < 1e-12 * abs(Kf).max()
    assert abs(Kf - Kf.T).max() == 0.0


def test_modal_boundary_matches_nodal_lattice():
    # the constrained modes are those whose lattice position is on the boundary
    n, p = 3, 4
    mm = synth.hex_mesh(n, p, basis="modal")
    mn = synth.hex_mesh(n, p, basis="nodal")
    cm = assembly.boundary_nodes(mm.l2g, p, mm.n_nodes, "modal")
    cn = assembly.boundary_nodes(mn.l2g, p, mn.n_nodes, "nodal")
    assert np.array_equal(cm, cn)


@pytest.mark.parametrize("p", [2, 4, 6])
def test_injection_galerkin_is_principal_submatrix(p):
    m = synth.hex_mesh(3, p, perturb=0.1, seed=3, basis="modal")
    H = hierarchy.build(m.coords, m.l2g, p, 2.0, hierarchy.Options(basis="modal", coarse_max=10))
    for lv, nxt in zip(H.levels[:-1], H.levels[1:]):
        if lv.collect is None:
            break
        P = lv.P.tocsr()
        assert np.all(P.data == 1.0) and np.all(np.diff(P.indptr) <= 1)
        assert P.nnz == lv.collect.size
        sub = lv.A[lv.collect][:, lv.collect]
        assert (abs(sub - nxt.A)).max() == 0.0


@pytest.mark.parametrize("p,q", [(4, 2), (6, 3)])
def test_modal_coarse_operator_is_direct_assembly(p, q):
    # nested hierarchical spaces: the kept modes of the order-p operator are
    # the order-q operator on the same geometry (same quadrature rule)
    n = 2
    mp = synth.hex_mesh(n, p, perturb=0.1, seed=5, basis="modal")
    mq = synth.hex_mesh(n, q, perturb=0.1, seed=5, basis="modal")
    Ap, cons = assembly.assemble(mp.coords, mp.l2g, p, 3.0, basis="modal")
    Aq, _ = assembly.assemble(mq.coords, mq.l2g, q, 3.0, nq=p + 2, bc="none", basis="modal")
    collect, l2g_nx, P = ptransfer.p_level(mp.l2g, p, q, mp.n_nodes, ~cons, "modal")
    # coarse id -> order-q mesh id through the kept local modes
    keep = ptransfer.extract_next_dof(p, q, "modal")
    qid = np.full(collect.size, -1, dtype=np.int64)
    for e in range(mp.n_elem):
        for a, loc in enumerate(keep):
            c = l2g_nx[e, a]
            if c >= 0:
                qid[c] = mq.l2g[e, a]
    Ac = (P.T @ Ap @ P).tocsr()
    ref = Aq[qid][:, qid]
    assert np.max(np.abs((Ac - ref).toarray())) <= 1e-13 * abs(ref).max()


def _manufactured(basis_name, n, p, lam):
    m = synth.hex_mesh(n, p, perturb=0.1, seed=7, basis=basis_name)
    A, cons = assembly.assemble(m.coords, m.l2g, p, lam, basis=basis_name)
    xq = assembly.quadrature_points(m.coords, m.l2g, p, basis=basis_name)
    fq = (lam + 3 * math.pi ** 2) * np.prod(np.sin(math.pi * xq), axis=2)
    b = assembly.load_vector(m.coords, m.l2g, p, fq, cons, basis=basis_name)
    u = spla.spsolve(A.tocsc(), b)
    return m, u


@pytest.mark.parametrize("n,p", [(2, 3), (2, 4)])
def test_modal_and_nodal_solutions_are_the_same_function(n, p):
    lam = 2.0
    mn, un = _manufactured("nodal", n, p, lam)
    mm, um = _manufactured("modal", n, p, lam)
    xg, _ = basis.gll_points(p)
    V = basis.modal_eval(p, xg)                      # [mode, gll point]
    for e in range(mn.n_elem):
        c = um[mm.l2g[e]].reshape(p + 1, p + 1, p + 1)
        at_gll = np.einsum("ijk,ia,jb,kc->abc", c, V, V, V).ravel()
        assert np.max(np.abs(at_gll - un[mn.l2g[e]])) < 1e-11 * np.max(np.abs(un))


def test_modal_hierarchy_solves():
    m = synth.hex_mesh(3, 4, perturb=0.1, seed=2, basis="modal")
    H = hierarchy.build(m.coords, m.l2g, 4, 10.0, hierarchy.Options(basis="modal", coarse_max=50))
    from oracle import krylov
    b = synth.normal_rhs(m.n_nodes, 3)
    r = krylov.giamg_pcg(H, b, tol=1e-10, maxit=1000)
    x = spla.spsolve(H.levels[0].A.tocsc(), b)
    assert r.converged
    assert np.linalg.norm(r.x - x) <= 1e-8 * np.linalg.norm(x)
