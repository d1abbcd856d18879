"""Pins of the oracle's fine-level assembly (problem of Section 3.1).

* all-node pattern size: the pattern of a structured mesh is the tensor cube
  of the 1-D pattern, nnz = (n (p+1)^2 - (n-1))^3, and 2 x 2 x 2 order-1
  elements give Table 1's coarsest 27 rows / 343 nonzeros;
* uniform meshes: the 3-D operator equals the Kronecker sum of 1-D operators
  built here from exact polynomial integration (closed-form GLL nodes);
* perturbed meshes: 1^T M 1 is the volume, K 1 = 0, bitwise symmetry;
* distorted elements (what pins the inverse Jacobian off the axis-aligned
  case): the patch test -- a globally linear u lies in the trilinear-mapped
  Q_p space, so K u vanishes on every row whose basis function vanishes on
  the boundary, exactly, because |J| J^-T is polynomial in the reference
  coordinates and p + 2 Gauss points integrate it; invariance of A under a
  rigid rotation of the mesh; the manufactured-solution rate p + 1 on
  perturbed meshes;
* Dirichlet structure and the manufactured-solution convergence rate.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import Polynomial

import synth
from oracle import assembly, ptransfer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

CLOSED_GLL = {1: [-1.0, 1.0], 2: [-1.0, 0.0, 1.0],
              3: [-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0],
              4: [-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0]}


def _lagrange_polys(nodes):
    out = []
    for i, xi in enumerate(nodes):
        others = [x for j, x in enumerate(nodes) if j != i]
        poly = Polynomial.fromroots(others)
        out.append(poly / poly(xi))
    return out


def _one_d(n, p):
    """Global 1-D mass and stiffness on [0, 1], n elements of order p, by
    exact integration of products of Lagrange polynomials."""
    polys = _lagrange_polys(CLOSED_GLL[p])
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
    for e in range(n):
        s = slice(e * p, e * p + p + 1)
        M[s, s] += Me
        K[s, s] += Ke
    return M, K


@pytest.mark.parametrize("n,p", [(1, 1), (2, 1), (3, 2), (2, 4), (4, 3)])
def test_all_node_pattern_formula(n, p):
    m = synth.hex_mesh(n, p)
    assert assembly.all_node_pattern_nnz(m.l2g, m.n_nodes) == (n * (p + 1) ** 2 - (n - 1)) ** 3


def test_table1_coarsest_level_pin():
    rows = [l for l in open(os.path.join(GOLDEN, "table1_giamg_hierarchy.txt"))
            if l.strip() and not l.startswith("#")]
    order, nel, levels, crow, cnnz = map(int, rows[0].split())
    assert len(ptransfer.p_schedule(order)) == levels
    m = synth.hex_mesh(nel, 1)
    assert m.n_nodes == crow
    assert assembly.all_node_pattern_nnz(m.l2g, m.n_nodes) == cnnz
    A, _ = assembly.assemble(m.coords, m.l2g, 1, 1.0, bc="none")
    assert A.shape == (crow, crow) and A.nnz == cnnz


def test_table1_hierarchy_with_boundary_kept():
    """The whole p-hierarchy on Table 1's mesh: with the constrained nodes
    kept on the coarse levels, p = 8 -> 4 -> 2 -> 1 gives 4 levels whose
    coarsest has 27 rows and 343 nonzeros, as printed; the default reading
    (free nodes only) leaves 1 row there."""
    from oracle import hierarchy
    rows = [l for l in open(os.path.join(GOLDEN, "table1_giamg_hierarchy.txt"))
            if l.strip() and not l.startswith("#")]
    order, nel, levels, crow, cnnz = map(int, rows[0].split())
    m = synth.hex_mesh(nel, order, perturb=0.1, seed=3)
    opts = hierarchy.Options(smoother="chebyshev", degree=3, keep_boundary=True)
    H = hierarchy.build(m.coords, m.l2g, order, 1.0, opts)
    assert len(H.levels) == levels and [lv.order for lv in H.levels] == [8, 4, 2, 1]
    assert [lv.A.shape[0] for lv in H.levels] == [(nel * q + 1) ** 3 for q in (8, 4, 2, 1)]
    assert H.levels[-1].A.shape == (crow, crow) and H.levels[-1].A.nnz == cnnz
    # every coarse operator is symmetric positive definite
    for lv in H.levels[1:]:
        D = lv.A.toarray()
        assert np.max(np.abs(D - D.T)) <= 1e-13 * np.max(np.abs(D))
        assert np.linalg.eigvalsh(D).min() > 0
    H0 = hierarchy.build(m.coords, m.l2g, order, 1.0, hierarchy.Options(smoother="chebyshev", degree=3))
    assert H0.levels[-1].A.shape == (1, 1)


@pytest.mark.parametrize("n,p,lam", [(2, 1, 1.0), (3, 2, 0.5), (2, 3, 10.0)])
def test_kronecker_sum_uniform(n, p, lam):
    m = synth.hex_mesh(n, p)
    A, _ = assembly.assemble(m.coords, m.l2g, p, lam, bc="none")
    M1, K1 = _one_d(n, p)
    ref = (np.kron(np.kron(K1, M1), M1) + np.kron(np.kron(M1, K1), M1)
           + np.kron(np.kron(M1, M1), K1) + lam * np.kron(np.kron(M1, M1), M1))
    D = A.toarray()
    assert np.max(np.abs(D - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_q1_uniform_stencil_closed_form():
    # interior Q1 Laplacian stencil on spacing h: centre 8h/3, neighbours
    # along an axis 0, across a face diagonal -h/6, across a body diagonal -h/12
    n = 4
    h = 1.0 / n
    m = synth.hex_mesh(n, 1)
    A, _ = assembly.assemble(m.coords, m.l2g, 1, 0.0, bc="none")
    L = n + 1
    c = (2 * L + 2) * L + 2
    row = A.getrow(c).toarray().ravel()
    assert abs(row[c] - 8 * h / 3) < 1e-15
    assert abs(row[c + 1]) < 1e-15
    assert abs(row[c + L + 1] + h / 6) < 1e-15
    assert abs(row[c + L * L + L + 1] + h / 12) < 1e-15


@pytest.mark.parametrize("n,p", [(3, 2), (2, 4), (2, 6)])
def test_perturbed_volume_nullspace_symmetry(n, p):
    m = synth.hex_mesh(n, p, perturb=0.2, seed=7)
    A1, _ = assembly.assemble(m.coords, m.l2g, p, 1.0, bc="none")
    A0, _ = assembly.assemble(m.coords, m.l2g, p, 0.0, bc="none")
    one = np.ones(m.n_nodes)
    M = A1 - A0
    assert abs(one @ (M @ one) - 1.0) < 1e-13
    assert np.max(np.abs(A0 @ one)) < 1e-12
    assert (A1 - A1.T).nnz == 0 or np.max(np.abs((A1 - A1.T).data)) == 0.0


def test_dirichlet_structure():
    n, p = 3, 2
    m = synth.hex_mesh(n, p, perturb=0.1, seed=3)
    A, cons = assembly.assemble(m.coords, m.l2g, p, 1.0)
    L = n * p + 1
    assert cons.sum() == L ** 3 - (L - 2) ** 3
    ci = np.nonzero(cons)[0]
    for i in ci[:20]:
        row = A.getrow(i)
        assert row.nnz == 1 and row.indices[0] == i and row.data[0] == 1.0
    # no free row stores a constrained column
    Af = A[~cons][:, cons]
    assert Af.nnz == 0
    # pin mode constrains node 0 only
    Ap, consp = assembly.assemble(m.coords, m.l2g, p, 0.0, bc="pin", pin=0)
    assert consp.sum() == 1 and consp[0]


def _nodal_error(n, p, lam):
    m = synth.hex_mesh(n, p)
    A, cons = assembly.assemble(m.coords, m.l2g, p, lam)
    xq = assembly.quadrature_points(m.coords, m.l2g, p)
    f = (lam + 3 * math.pi ** 2) * np.prod(np.sin(math.pi * xq), axis=2)
    b = assembly.load_vector(m.coords, m.l2g, p, f, cons)
    u = spla.spsolve(A.tocsc(), b)
    # true GLL node positions on the uniform mesh, from closed forms
    g = np.array(CLOSED_GLL[p])
    lat = []
    for e in range(n):
        lat.extend(((e + (g[:-1] + 1) / 2) / n).tolist())
    lat.append(1.0)
    lat = np.array(lat)
    X, Y, Z = np.meshgrid(lat, lat, lat, indexing="ij")
    ue = (np.sin(math.pi * X) * np.sin(math.pi * Y) * np.sin(math.pi * Z)).ravel()
    return np.max(np.abs(u - ue))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_manufactured_solution_rate(p):
    e1 = _nodal_error(2, p, 1.0)
    e2 = _nodal_error(4, p, 1.0)
    rate = math.log2(e1 / e2)
    assert rate > p + 0.6, (e1, e2, rate)


def _gll_node_positions(m, p):
    """Physical position of every node: its element's trilinear map of the
    eight corners evaluated at the node's closed-form GLL reference point.
    Shared nodes get the same point from every element that holds them (a
    trilinear map restricted to a face is fixed by the face's corners);
    checked."""
    g = np.array(CLOSED_GLL[p])
    pos = np.full((m.n_nodes, 3), np.nan)
    corners = [m.l2g[:, (p + 1) ** 2 * (cx * p) + (p + 1) * (cy * p) + cz * p]
               for cx in (0, 1) for cy in (0, 1) for cz in (0, 1)]
    X = np.stack([m.coords[c] for c in corners], axis=1)          # [E, 8, 3]
    for i in range(p + 1):
        for j in range(p + 1):
            for k in range(p + 1):
                t = (np.array([g[i], g[j], g[k]]) + 1.0) / 2.0
                w = [((t[0] if cx else 1 - t[0]) * (t[1] if cy else 1 - t[1])
                      * (t[2] if cz else 1 - t[2]))
                     for cx in (0, 1) for cy in (0, 1) for cz in (0, 1)]
                x = np.einsum("c,eca->ea", np.array(w), X)
                ids = m.l2g[:, (p + 1) ** 2 * i + (p + 1) * j + k]
                seen = ~np.isnan(pos[ids, 0])
                assert np.allclose(pos[ids[seen]], x[seen], rtol=0, atol=1e-14)
                pos[ids] = x
    assert not np.isnan(pos).any()
    return pos


@pytest.mark.parametrize("p,perturb,seed", [(1, 0.2, 11), (2, 0.15, 12), (3, 0.2, 13),
                                            (4, 0.1, 14), (4, 0.2, 15)])
def test_patch_test_distorted(p, perturb, seed):
    """K u = 0 on the rows of nodes off the boundary for u = a.x + c."""
    m = synth.hex_mesh(3, p, perturb=perturb, seed=seed)
    K, _ = assembly.assemble(m.coords, m.l2g, p, 0.0, bc="none")
    x = _gll_node_positions(m, p)
    u = x @ np.array([0.7, -1.3, 2.1]) + 0.4
    Ku = K @ u
    bnd = assembly.boundary_nodes(m.l2g, p, m.n_nodes)
    scale = abs(K) @ abs(u)
    interior = ~bnd
    assert interior.sum() == (3 * p - 1) ** 3
    assert np.max(np.abs(Ku[interior]) / scale[interior]) < 1e-13
    # the boundary rows carry the flux of a and are not zero: the check is
    # not vacuous
    assert np.max(np.abs(Ku[bnd]) / scale[bnd]) > 1e-3


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rotation_invariance_distorted(p):
    """A rigid motion of the mesh leaves K and M unchanged."""
    m = synth.hex_mesh(2, p, perturb=0.2, seed=21 + p)
    th = np.array([0.3, -1.1, 0.7])
    cx, cy, cz = np.cos(th)
    sx, sy, sz = np.sin(th)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    Q = Rz @ Ry @ Rx
    moved = m.coords @ Q.T + np.array([0.5, -2.0, 1.0])
    A, _ = assembly.assemble(m.coords, m.l2g, p, 3.0, bc="none")
    B, _ = assembly.assemble(moved, m.l2g, p, 3.0, bc="none")
    assert (A.indptr == B.indptr).all() and (A.indices == B.indices).all()
    assert np.max(np.abs(A.data - B.data)) <= 1e-13 * np.max(np.abs(A.data))


def _refined(coarse, r, p):
    """The mesh that splits every element of ``coarse`` into r^3: its
    vertices are the images of the uniform r-times finer grid under the
    coarse mesh's piecewise trilinear map, so each fine element is exactly
    the image of a sub-cube (a trilinear map restricted to a sub-box is
    trilinear) and the discrete spaces are nested."""
    n0 = coarse.n
    V = coarse.vertices.reshape(n0 + 1, n0 + 1, n0 + 1, 3)
    fine = synth.hex_mesh(n0 * r, p)
    y = fine.coords                                 # uniform lattice positions
    e = np.minimum(np.floor(y * n0).astype(int), n0 - 1)
    t = y * n0 - e
    x = np.zeros_like(y)
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                w = ((t[:, 0] if cx else 1 - t[:, 0]) * (t[:, 1] if cy else 1 - t[:, 1])
                     * (t[:, 2] if cz else 1 - t[:, 2]))
                x += w[:, None] * V[e[:, 0] + cx, e[:, 1] + cy, e[:, 2] + cz]
    fine.coords = x
    return fine


def _nodal_error_on(m, p, lam):
    A, cons = assembly.assemble(m.coords, m.l2g, p, lam)
    xq = assembly.quadrature_points(m.coords, m.l2g, p)
    f = (lam + 3 * math.pi ** 2) * np.prod(np.sin(math.pi * xq), axis=2)
    b = assembly.load_vector(m.coords, m.l2g, p, f, cons)
    u = spla.spsolve(A.tocsc(), b)
    x = _gll_node_positions(m, p)
    ue = np.prod(np.sin(math.pi * x), axis=1)
    return np.max(np.abs(u - ue))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_manufactured_solution_rate_perturbed(p):
    """Error at the nodes of the discrete solution on a perturbed mesh and
    on its uniform refinement (every element split in eight): the rate of
    an order-p method, p + 1."""
    coarse = synth.hex_mesh(2, p, perturb=0.15, seed=31)
    e1 = _nodal_error_on(coarse, p, 1.0)
    e2 = _nodal_error_on(_refined(coarse, 2, p), p, 1.0)
    rate = math.log2(e1 / e2)
    assert rate > p + 0.6, (e1, e2, rate)
