"""Fine-level operator A = K + lambda M for hexahedra of order p (oracle).

Problem statement: the Helmholtz equation -lap u + lambda u = f on the unit
cube with homogeneous Dirichlet data (Section 3.1, Helmholtz operator); the
pressure-Poisson case is lambda = 0 (Section 3.2).  The paper assembles with
Nektar++; the readings below replace that:

* basis: tensor-product Lagrange on GLL points ("nodal"), or the
  appendix's hierarchical modal basis ("modal": 1-D modes (1-a)/2, (1+a)/2,
  then bubbles); local index (p+1)^2 i + (p+1) j + k with i along x
  (appendix ordering).  The vertex modes/nodes at a = -1 and a = +1 have
  local index 0 and p (nodal) or 0 and 1 (modal);
* geometry: the trilinear map of the element's eight corner nodes;
* quadrature: Gauss-Legendre with p+2 points per direction, consistent mass;
* pattern: (r, c) is stored when r and c belong to a common element
  ("share an element"), with explicit zeros kept;
* boundary conditions: a node on a face owned by exactly one element is
  constrained (Dirichlet mode), or only the pinned node is (pin mode).  A
  constrained node's row and column are replaced by the identity: the row
  holds only its unit diagonal and no free row stores the column.

TEST INFRASTRUCTURE ONLY.
"""
import numpy as np
import scipy.sparse as sp

from .basis import (gll_points, gauss_points, lagrange_eval, lagrange_deriv, modal_eval,
                    modal_deriv)

BASES = ("nodal", "modal")


def local_index(p: int, i, j, k):
    return (p + 1) * (p + 1) * i + (p + 1) * j + k


def ends(p: int, basis: str = "nodal"):
    """1-D local indices of the modes/nodes that are one at a = -1 and a = +1."""
    if basis not in BASES:
        raise ValueError(basis)
    return (0, p) if basis == "nodal" else (0, 1)


def corner_local_indices(p: int, basis: str = "nodal") -> np.ndarray:
    """Local indices of the 8 corners, corner c = 4 cx + 2 cy + cz."""
    e = ends(p, basis)
    out = []
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                out.append(local_index(p, e[cx], e[cy], e[cz]))
    return np.array(out)


def face_local_indices(p: int, basis: str = "nodal"):
    """The six faces of the reference hexahedron: the local indices of the
    modes/nodes not vanishing on each face, in (A, B) row-major order."""
    r = np.arange(p + 1)
    A, B = np.meshgrid(r, r, indexing="ij")
    A, B = A.ravel(), B.ravel()
    faces = []
    for fixed in ends(p, basis):
        faces.append(local_index(p, fixed, A, B))
        faces.append(local_index(p, A, fixed, B))
        faces.append(local_index(p, A, B, fixed))
    return faces


def boundary_nodes(l2g: np.ndarray, p: int, n_nodes: int, basis: str = "nodal") -> np.ndarray:
    """Boolean mask: node (mode) lies on a face that belongs to exactly one
    element; faces are told apart by their four corner ids."""
    faces = face_local_indices(p, basis)
    lo, hi = ends(p, basis)
    cpos = [lo * (p + 1) + lo, lo * (p + 1) + hi, hi * (p + 1) + lo, hi * (p + 1) + hi]
    keys = []
    members = []
    for f in faces:
        corners = l2g[:, f[cpos]].astype(np.int64)
        keys.append(np.sort(corners, axis=1))
        members.append(l2g[:, f])
    keys = np.concatenate(keys, axis=0)
    members = np.concatenate(members, axis=0)
    _, inv, cnt = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    on_bnd = cnt[inv.ravel()] == 1
    mask = np.zeros(n_nodes, dtype=bool)
    mask[members[on_bnd].ravel()] = True
    return mask


def constrained_mask(l2g, p, n_nodes, bc="dirichlet", pin=0, basis="nodal"):
    if bc == "dirichlet":
        return boundary_nodes(l2g, p, n_nodes, basis)
    if bc == "pin":
        m = np.zeros(n_nodes, dtype=bool)
        m[pin] = True
        return m
    if bc == "none":
        return np.zeros(n_nodes, dtype=bool)
    raise ValueError(bc)


def _reference_tables(p: int, nq: int, basis: str = "nodal"):
    """Basis values/gradients and trilinear-map derivatives at the tensor
    Gauss points (x slowest)."""
    xg, wg = gauss_points(nq)
    if basis == "nodal":
        xn, _ = gll_points(p)
        L = lagrange_eval(xn, xg)       # [p+1, nq]
        D = lagrange_deriv(xn, xg)
    else:
        L = modal_eval(p, xg)
        D = modal_deriv(p, xg)
    nl = (p + 1) ** 3
    Q = nq ** 3
    phi = np.zeros((nl, Q))
    dphi = np.zeros((nl, Q, 3))
    for i in range(p + 1):
        for j in range(p + 1):
            for k in range(p + 1):
                a = local_index(p, i, j, k)
                phi[a] = np.einsum("x,y,z->xyz", L[i], L[j], L[k]).ravel()
                dphi[a, :, 0] = np.einsum("x,y,z->xyz", D[i], L[j], L[k]).ravel()
                dphi[a, :, 1] = np.einsum("x,y,z->xyz", L[i], D[j], L[k]).ravel()
                dphi[a, :, 2] = np.einsum("x,y,z->xyz", L[i], L[j], D[k]).ravel()
    w = np.einsum("x,y,z->xyz", wg, wg, wg).ravel()
    X, Y, Z = np.meshgrid(xg, xg, xg, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    # trilinear shape functions N_c and their derivatives
    N = np.zeros((8, Q))
    dN = np.zeros((8, Q, 3))
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                c = 4 * cx + 2 * cy + cz
                s = np.array([2 * cx - 1, 2 * cy - 1, 2 * cz - 1], dtype=float)
                f = (1.0 + s[None, :] * xi) / 2.0     # [Q, 3]
                N[c] = f[:, 0] * f[:, 1] * f[:, 2]
                dN[c, :, 0] = s[0] / 2.0 * f[:, 1] * f[:, 2]
                dN[c, :, 1] = f[:, 0] * s[1] / 2.0 * f[:, 2]
                dN[c, :, 2] = f[:, 0] * f[:, 1] * s[2] / 2.0
    return phi, dphi, w, N, dN


def element_geometry(coords, l2g, p, N, dN, basis="nodal"):
    """Jacobian J[e, q, a, d] = d x_a / d xi_d and det J per element and point."""
    X = coords[l2g[:, corner_local_indices(p, basis)]]   # [E, 8, 3]
    J = np.einsum("eca,cqd->eqad", X, dN)
    det = np.linalg.det(J)
    xq = np.einsum("eca,cq->eqa", X, N)
    return J, det, xq


def element_matrices(coords, l2g, p, nq, lam, basis="nodal"):
    """Element matrices K_e + lam M_e, symmetrised by mirroring the upper
    triangle so the assembled matrix is bitwise symmetric.  Yields chunks
    (element ids, matrices)."""
    phi, dphi, w, N, dN = _reference_tables(p, nq, basis)
    E = l2g.shape[0]
    nl = (p + 1) ** 3
    iu = np.triu_indices(nl, 1)
    chunk = max(1, int(2e7 // (nl * nl + nl * phi.shape[1] * 3)))
    for e0 in range(0, E, chunk):
        e1 = min(E, e0 + chunk)
        J, det, _ = element_geometry(coords, l2g[e0:e1], p, N, dN, basis)
        if np.any(det <= 0):
            raise ValueError("non-positive Jacobian determinant")
        Jinv = np.linalg.inv(J)                                  # [e,q,d,a]
        g = np.einsum("eqda,iqd->eqia", Jinv, dphi)              # physical grads
        wd = w[None, :] * det                                    # [e,q]
        ne = e1 - e0
        # K_e = sum over points and directions of w |J| grad phi_i . grad phi_j
        G = g.transpose(0, 2, 1, 3).reshape(ne, nl, -1)          # [e, i, q*3]
        Gw = (g * wd[:, :, None, None]).transpose(0, 2, 1, 3).reshape(ne, nl, -1)
        K = Gw @ G.transpose(0, 2, 1)
        # M_e = sum over points of w |J| phi_i phi_j
        Pw = phi[None, :, :] * wd[:, None, :]                     # [e, i, q]
        M = Pw @ phi.T[None, :, :]
        A = K + lam * M
        A[:, iu[1], iu[0]] = A[:, iu[0], iu[1]]
        yield np.arange(e0, e1), A


def assemble(coords, l2g, p, lam, bc="dirichlet", pin=0, nq=None, basis="nodal"):
    """Assembled CSR matrix (float64, int32 indices) and the constrained mask."""
    n_nodes = coords.shape[0]
    nq = p + 2 if nq is None else nq
    cons = constrained_mask(l2g, p, n_nodes, bc, pin, basis)
    nl = (p + 1) ** 3
    rows_l, cols_l, vals_l = [], [], []
    for eids, Ae in element_matrices(coords, l2g, p, nq, lam, basis):
        g = l2g[eids].astype(np.int64)
        rows_l.append(np.repeat(g, nl, axis=1).ravel())
        cols_l.append(np.tile(g, (1, nl)).ravel())
        vals_l.append(Ae.reshape(len(eids), -1).ravel())
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l)
    vals = np.concatenate(vals_l)
    return _coo_to_csr_with_bc(rows, cols, vals, n_nodes, cons), cons


def _coo_to_csr_with_bc(rows, cols, vals, n, cons):
    """Sum duplicates in element order, keep the symbolic pattern, then
    apply the identity rows/columns of constrained nodes."""
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key_s = key[order]
    uniq, start = np.unique(key_s, return_index=True)
    summed = np.add.reduceat(vals[order], start) if len(vals) else np.zeros(0)
    r = uniq // n
    c = uniq % n
    keep = ~cons[r] & ~cons[c]
    r, c, v = r[keep], c[keep], summed[keep]
    ci = np.nonzero(cons)[0]
    r = np.concatenate([r, ci])
    c = np.concatenate([c, ci])
    v = np.concatenate([v, np.ones(len(ci))])
    return csr_from_sorted_or_not(r, c, v, n, n)


def csr_from_sorted_or_not(r, c, v, nr, nc):
    """CSR with sorted column indices and explicit zeros kept."""
    key = np.asarray(r, dtype=np.int64) * nc + np.asarray(c, dtype=np.int64)
    order = np.argsort(key, kind="stable")
    r = np.asarray(r)[order]
    c = np.asarray(c)[order]
    v = np.asarray(v, dtype=np.float64)[order]
    indptr = np.zeros(nr + 1, dtype=np.int64)
    np.add.at(indptr, r + 1, 1)
    indptr = np.cumsum(indptr)
    M = sp.csr_matrix((v, c.astype(np.int32), indptr), shape=(nr, nc))
    M.has_sorted_indices = True
    return M


def quadrature_points(coords, l2g, p, nq=None, basis="nodal"):
    """Physical coordinates of the tensor Gauss points, [E, nq^3, 3]."""
    nq = p + 2 if nq is None else nq
    _, _, _, N, dN = _reference_tables(p, nq, basis)
    _, _, xq = element_geometry(coords, l2g, p, N, dN, basis)
    return xq


def load_vector(coords, l2g, p, fq, cons, nq=None, basis="nodal"):
    """b_i = sum over elements of the quadrature of f phi_i, with f given at
    the element quadrature points (fq: [E, nq^3]); b = 0 on constrained
    nodes (homogeneous Dirichlet data)."""
    nq = p + 2 if nq is None else nq
    phi, _, w, N, dN = _reference_tables(p, nq, basis)
    _, det, _ = element_geometry(coords, l2g, p, N, dN, basis)
    be = np.einsum("iq,eq,eq->ei", phi, w[None, :] * det, fq)
    b = np.zeros(coords.shape[0])
    np.add.at(b, l2g.ravel(), be.ravel())
    b[cons] = 0.0
    return b


def all_node_pattern_nnz(l2g, n_nodes) -> int:
    """Number of (r, c) pairs that share an element, counting every node."""
    nl = l2g.shape[1]
    g = l2g.astype(np.int64)
    key = (np.repeat(g, nl, axis=1) * n_nodes + np.tile(g, (1, nl))).ravel()
    return int(np.unique(key).size)
