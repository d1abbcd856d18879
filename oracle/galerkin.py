"""Galerkin coarse operators A_c = R A_f P with R = P^T (oracle).

Section 2.1 (after Algorithm 1): the coarse operator is the Galerkin product
computed and stored at setup.  Reading: the structure of a product is its
full symbolic structure (an entry exists when some term contributes, even if
the terms cancel), columns ascending; values are R (A P) summed in the
natural order of scipy's row-by-row product.

TEST INFRASTRUCTURE ONLY.
"""
import numpy as np
import scipy.sparse as sp


def pattern_of(M: sp.csr_matrix) -> sp.csr_matrix:
    """Same structure, all stored values replaced by 1.0 (explicit zeros kept)."""
    S = sp.csr_matrix((np.ones(M.nnz), M.indices.copy(), M.indptr.copy()),
                      shape=M.shape)
    return S


def symbolic_product(A: sp.csr_matrix, B: sp.csr_matrix) -> sp.csr_matrix:
    """Structure of A B: products of positive ones never cancel."""
    S = (pattern_of(A) @ pattern_of(B)).tocsr()
    S.sort_indices()
    S.data[:] = 1.0
    return S


def values_on_pattern(pattern: sp.csr_matrix, numeric: sp.csr_matrix) -> sp.csr_matrix:
    """Matrix with ``pattern``'s structure and ``numeric``'s values (0.0 where
    numeric has no stored entry).  numeric's structure must be a subset."""
    pattern = pattern.tocsr()
    numeric = numeric.tocsr()
    numeric.sum_duplicates()
    nr, nc = pattern.shape
    pr = np.repeat(np.arange(nr, dtype=np.int64), np.diff(pattern.indptr))
    pkey = pr * nc + pattern.indices
    nrr = np.repeat(np.arange(nr, dtype=np.int64), np.diff(numeric.indptr))
    nkey = nrr * nc + numeric.indices
    order = np.argsort(pkey)
    pos = np.searchsorted(pkey[order], nkey)
    assert np.all(pkey[order][pos] == nkey), "numeric entry outside pattern"
    vals = np.zeros(pattern.nnz)
    vals[order[pos]] = numeric.data
    out = sp.csr_matrix((vals, pattern.indices.copy(), pattern.indptr.copy()),
                        shape=pattern.shape)
    out.has_sorted_indices = True
    return out


def transpose(P: sp.csr_matrix) -> sp.csr_matrix:
    R = P.T.tocsr()
    R.sort_indices()
    return R


def rap(R: sp.csr_matrix, A: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """A_c = R (A P) on the symbolic structure of R A P."""
    S = symbolic_product(R, symbolic_product(A, P))
    AP = A @ P
    num = R @ AP
    return values_on_pattern(S, num)
