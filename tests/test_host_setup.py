"""Host-side setup stages of the library against the oracle (CPU only).

Integer work bit-exact: constrained-node masks, CSR structures of A and P,
next-level element maps, aggregates.  Floating point within tolerances set
by the arithmetic: assembled values (the same quadrature summed in another
order: a few ulps of the largest term) and transfer values.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import assembly, ptransfer, sa
from paper_2512_15121_amd import giamg


def _csr(rp, ci, val, shape):
    return sp.csr_matrix((val, ci, rp), shape=shape)


@pytest.mark.parametrize("n,p,pert", [(3, 2, 0.1), (2, 4, 0.2), (3, 3, 0.0), (2, 6, 0.15)])
def test_boundary_mask_bitexact(n, p, pert):
    m = synth.hex_mesh(n, p, perturb=pert, seed=1)
    ref = assembly.boundary_nodes(m.l2g, p, m.n_nodes)
    got = giamg.host_boundary(m.l2g, p, m.n_nodes)
    assert np.array_equal(ref, got)


@pytest.mark.parametrize("n,p,lam,bc", [(3, 2, 1.0, "dirichlet"), (2, 4, 10.0, "dirichlet"),
                                        (3, 3, 0.0, "pin"), (2, 5, 0.3, "dirichlet"),
                                        (1, 1, 1.0, "pin"), (4, 1, 2.0, "dirichlet")])
def test_assembly_against_oracle(n, p, lam, bc):
    m = synth.hex_mesh(n, p, perturb=0.15, seed=3)
    A, _ = assembly.assemble(m.coords, m.l2g, p, lam, bc=bc)
    rp, ci, val, shape = giamg.host_assemble(m.coords, m.l2g, p, lam, bc=bc)
    assert np.array_equal(rp, A.indptr) and np.array_equal(ci, A.indices)
    # |a_ij - a_ij^o| <= 1e-13 max|a|: both sides evaluate the same quadrature
    scale = np.abs(A.data).max()
    assert np.max(np.abs(val - A.data)) <= 1e-13 * scale
    # bitwise symmetric on the library side as well
    G = _csr(rp, ci, val, shape)
    assert (G != G.T).nnz == 0


def test_assembly_rejects_inverted_element():
    m = synth.hex_mesh(2, 1)
    l2g = m.l2g.copy()
    l2g[0] = l2g[0][[4, 5, 6, 7, 0, 1, 2, 3]]   # mirror element 0 in x
    with pytest.raises(giamg.GiamgError) as e:
        giamg.host_assemble(m.coords, l2g, 1, 1.0)
    assert "Jacobian" in str(e.value)


@pytest.mark.parametrize("n,p,q,bc", [(3, 2, 1, "dirichlet"), (3, 4, 2, "dirichlet"),
                                      (2, 6, 3, "dirichlet"), (2, 4, 2, "pin"), (3, 5, 1, "dirichlet")])
def test_p_transfer_against_oracle(n, p, q, bc):
    m = synth.hex_mesh(n, p, perturb=0.1, seed=5)
    cons = assembly.constrained_mask(m.l2g, p, m.n_nodes, bc, 0)
    collect, l2g_nx, P = ptransfer.p_level(m.l2g, p, q, m.n_nodes, ~cons)
    nxt, nc, (rp, ci, val, shape) = giamg.host_p_transfer(m.l2g, p, q, m.n_nodes, ~cons)
    assert nc == collect.size and shape == P.shape
    assert np.array_equal(nxt, l2g_nx)
    assert np.array_equal(rp, P.indptr) and np.array_equal(ci, P.indices)
    assert np.max(np.abs(val - P.data)) <= 1e-14
    # second step on the coarse map (constrained entries are -1 there)
    if q > 1:
        r = ptransfer.p_schedule(q)[1]
        free2 = np.ones(nc, dtype=bool)
        c2, l2, P2 = ptransfer.p_level(l2g_nx, q, r, nc, free2)
        nx2, nc2, (rp2, ci2, val2, _) = giamg.host_p_transfer(nxt, q, r, nc, free2)
        assert nc2 == c2.size and np.array_equal(nx2, l2)
        assert np.array_equal(rp2, P2.indptr) and np.array_equal(ci2, P2.indices)
        assert np.max(np.abs(val2 - P2.data)) <= 1e-14


@pytest.mark.parametrize("n,seed", [(7, 0), (9, 12345), (10, 2 ** 63 + 7)])
def test_aggregation_against_oracle(n, seed):
    m = synth.hex_mesh(n, 1, perturb=0.1, seed=4)
    A, cons = assembly.assemble(m.coords, m.l2g, 1, 1.5)
    free = np.nonzero(~cons)[0]
    Af = A[free][:, free].tocsr()
    Af.sort_indices()
    agg_o, roots = sa.aggregate(Af, seed)
    P_o, _, _ = sa.smoothed_prolongation(Af, agg_o, roots.size)
    agg, na, (rp, ci, val, shape) = giamg.host_aggregate(Af.indptr, Af.indices, Af.data, seed)
    assert na == roots.size and np.array_equal(agg, agg_o)
    assert np.array_equal(rp, P_o.indptr) and np.array_equal(ci, P_o.indices)
    assert np.max(np.abs(val - P_o.data)) <= 1e-15


@pytest.mark.parametrize("n,seed,theta", [(8, 3, 0.05), (9, 77, 0.1)])
def test_aggregation_with_strength_threshold_against_oracle(n, seed, theta):
    """Strength threshold theta > 0 (the graph drops weak couplings): the
    library's aggregates and P equal the oracle's.  Both decide strength on
    the same host values; the test first checks that no coupling lies within
    1e-9 of the threshold, so the integer result does not hang on rounding."""
    m = synth.hex_mesh(n, 1, perturb=0.2, seed=5)
    A, cons = assembly.assemble(m.coords, m.l2g, 1, 0.3)
    free = np.nonzero(~cons)[0]
    Af = A[free][:, free].tocsr()
    Af.sort_indices()
    d = np.abs(Af.diagonal())
    C = Af.tocoo()
    off = C.row != C.col
    ratio = np.abs(C.data[off]) / np.sqrt(d[C.row[off]] * d[C.col[off]])
    assert np.min(np.abs(ratio - theta)) > 1e-9
    assert (ratio < theta).any() and (ratio >= theta).any()     # the threshold bites
    agg_o, roots = sa.aggregate(Af, seed, theta)
    agg0, roots0 = sa.aggregate(Af, seed, 0.0)
    assert not np.array_equal(agg_o, agg0)
    P_o, _, _ = sa.smoothed_prolongation(Af, agg_o, roots.size)
    agg, na, (rp, ci, val, shape) = giamg.host_aggregate(Af.indptr, Af.indices, Af.data, seed,
                                                         theta)
    assert na == roots.size and np.array_equal(agg, agg_o)
    assert np.array_equal(rp, P_o.indptr) and np.array_equal(ci, P_o.indices)
    assert np.max(np.abs(val - P_o.data)) <= 1e-15


# ---- modal basis (appendix ordering, injection transfers) ----------------
@pytest.mark.parametrize("n,p", [(3, 2), (2, 5)])
def test_modal_boundary_bitexact(n, p):
    m = synth.hex_mesh(n, p, perturb=0.1, seed=1, basis="modal")
    ref = assembly.boundary_nodes(m.l2g, p, m.n_nodes, "modal")
    got = giamg.host_boundary(m.l2g, p, m.n_nodes, basis="modal")
    assert np.array_equal(ref, got)


@pytest.mark.parametrize("n,p,lam,bc", [(3, 2, 1.0, "dirichlet"), (2, 4, 10.0, "dirichlet"),
                                        (2, 3, 0.0, "pin"), (2, 6, 0.5, "dirichlet")])
def test_modal_assembly_against_oracle(n, p, lam, bc):
    # library: Legendre closed forms of the modes; oracle: Jacobi polynomials
    m = synth.hex_mesh(n, p, perturb=0.15, seed=3, basis="modal")
    A, _ = assembly.assemble(m.coords, m.l2g, p, lam, bc=bc, basis="modal")
    rp, ci, val, shape = giamg.host_assemble(m.coords, m.l2g, p, lam, bc=bc, basis="modal")
    assert np.array_equal(rp, A.indptr) and np.array_equal(ci, A.indices)
    assert np.max(np.abs(val - A.data)) <= 1e-13 * np.abs(A.data).max()
    G = _csr(rp, ci, val, shape)
    assert (G != G.T).nnz == 0


@pytest.mark.parametrize("n,p,q", [(3, 4, 2), (2, 6, 3), (3, 3, 1), (2, 5, 2)])
def test_modal_p_transfer_is_injection(n, p, q):
    m = synth.hex_mesh(n, p, perturb=0.1, seed=5, basis="modal")
    cons = assembly.constrained_mask(m.l2g, p, m.n_nodes, "dirichlet", 0, "modal")
    collect, l2g_nx, P = ptransfer.p_level(m.l2g, p, q, m.n_nodes, ~cons, "modal")
    nxt, nc, (rp, ci, val, shape) = giamg.host_p_transfer(m.l2g, p, q, m.n_nodes, ~cons,
                                                          basis="modal")
    assert nc == collect.size and np.array_equal(nxt, l2g_nx)
    assert np.array_equal(rp, P.indptr) and np.array_equal(ci, P.indices)
    assert np.all(val == 1.0) and np.all(np.diff(rp) <= 1)


@pytest.mark.parametrize("n,p,q", [(2, 5, 4), (3, 6, 4), (2, 5, 3), (3, 4, 3)])
def test_nodal_non_divisor_transfer_against_oracle(n, p, q):
    # a coarse order that does not divide p: nearest-lattice numbering, and
    # interpolation from GLL points that are not fine points
    m = synth.hex_mesh(n, p, perturb=0.1, seed=6)
    cons = assembly.constrained_mask(m.l2g, p, m.n_nodes, "dirichlet", 0)
    collect, l2g_nx, P = ptransfer.p_level(m.l2g, p, q, m.n_nodes, ~cons)
    nxt, nc, (rp, ci, val, shape) = giamg.host_p_transfer(m.l2g, p, q, m.n_nodes, ~cons)
    assert nc == collect.size and np.array_equal(nxt, l2g_nx)
    assert np.array_equal(rp, P.indptr) and np.array_equal(ci, P.indices)
    assert np.max(np.abs(val - P.data)) <= 1e-14


def test_transfer_rejects_non_decreasing_order():
    m = synth.hex_mesh(2, 3, basis="nodal")
    with pytest.raises(giamg.GiamgError):
        giamg.host_p_transfer(m.l2g, 3, 3, m.n_nodes, np.ones(m.n_nodes, dtype=bool))


# ---- dense inverse of the coarsest operator --------------------------------
def _spd(n, seed, cond=1e3):
    """Symmetric positive definite test matrix with eigenvalues spread
    log-uniformly over [1, cond] in a random orthonormal basis."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.logspace(0.0, np.log10(cond), n)
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("n", [1, 2, 31, 63, 64, 65, 200, 721])
def test_coarse_inverse_against_lapack(n):
    """Sizes below and above the point where the factorisation splits its
    columns over threads.  The inverse is exactly symmetric, and A X = I and
    X equals LAPACK's inverse to the rounding error of a condition-1000
    system."""
    A = _spd(n, 100 + n)
    X = giamg.host_coarse_inverse(A)
    assert np.array_equal(X, X.T)
    assert np.max(np.abs(A @ X - np.eye(n))) <= 1e-11
    ref = np.linalg.inv(A)
    assert np.max(np.abs(X - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_coarse_inverse_reads_the_lower_triangle_only():
    A = _spd(90, 7)
    B = A.copy()
    B[np.triu_indices(90, 1)] = np.nan
    assert np.array_equal(giamg.host_coarse_inverse(A), giamg.host_coarse_inverse(B))


def test_coarse_inverse_closed_forms():
    # 1 x 1 and diagonal: the factor is the square root, the solves divide
    # by it twice (within two roundings of 1/d)
    assert giamg.host_coarse_inverse(np.array([[4.0]]))[0, 0] == 0.25
    d = np.linspace(0.5, 50.0, 70)
    X = giamg.host_coarse_inverse(np.diag(d))
    assert np.count_nonzero(X - np.diag(np.diag(X))) == 0
    assert np.max(np.abs(np.diag(X) * d - 1.0)) <= 4e-16
    # tridiagonal [-1, 2, -1]: (A^-1)_ij = min(i, j) (n + 1 - max(i, j)) / (n + 1)
    n = 80
    T = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    i = np.arange(1, n + 1)
    exact = np.minimum.outer(i, i) * (n + 1 - np.maximum.outer(i, i)) / (n + 1)
    assert np.max(np.abs(giamg.host_coarse_inverse(T) - exact)) <= 1e-11 * exact.max()


def test_coarse_inverse_of_table1_coarsest_operator():
    """Table 1's mesh with the boundary kept: the 27-row order-1 operator at
    the bottom of the p-hierarchy (oracle), inverted as the setup does."""
    from oracle import hierarchy
    m = synth.hex_mesh(2, 8, perturb=0.1, seed=3)
    H = hierarchy.build(m.coords, m.l2g, 8, 1.0,
                        hierarchy.Options(smoother="chebyshev", degree=3, keep_boundary=True))
    A = H.levels[-1].A.toarray()
    assert A.shape == (27, 27)
    X = giamg.host_coarse_inverse(A)
    assert np.max(np.abs(A @ X - np.eye(27))) <= 1e-12 * np.linalg.cond(A)


def test_coarse_inverse_rejects_indefinite_and_bad_sizes():
    for A in (np.array([[1.0, 2.0], [2.0, 1.0]]), np.zeros((100, 100)), np.array([[np.nan]]),
              -np.eye(70)):
        with pytest.raises(giamg.GiamgError) as e:
            giamg.host_coarse_inverse(A)
        assert e.value.code == giamg.EINVAL
    lib = giamg.library()
    buf = np.zeros(4)
    for n in (0, -1, 16385):   # rejected before any element is read
        assert lib.giamg_host_coarse_inverse(giamg._ptr(buf), n, giamg._ptr(buf)) == giamg.EINVAL
    with pytest.raises(ValueError):
        giamg.host_coarse_inverse(np.zeros((3, 4)))
