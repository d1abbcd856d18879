"""p-coarsening transfer operators (oracle, test infrastructure only).

Follows Section 2.2 (computation of the l2g map at each level):
Algorithm 2 (extract the element dofs kept at the next level), Algorithm 3
(collect the kept dofs over all elements and sort them), Algorithm 4 (the
next-level l2g map through the rank of each kept dof in the sorted
collection), and Section 2.4 / Algorithm 7 (prolongation as COO triples,
sorted, duplicates removed).  With the modal basis (appendix ordering)
Algorithm 2 keeps the local modes i, j, k <= q, which are the order-q modes
themselves, and P injects them (entries 1.0).  The nodal variant (footnote
to Algorithm 7; Introduction) replaces the injected 1.0 by the lower-order
basis evaluated at the higher-order nodes.

Readings where the paper is silent:
* schedule: q = p / (smallest prime factor of p), so the coarse order
  divides the fine one (8 -> 4 -> 2 -> 1 gives Table 1's four levels);
* the coarse local node (a, b, c) is kept at the fine local node
  (pos(a), pos(b), pos(c)) for nodal GLL bases, pos(a) = floor((2 a p + q) /
  (2 q)) (the nearest lattice position; a p / q when q divides p).  The kept
  fine node only numbers the coarse node; P interpolates from the order-q
  GLL points whether or not they coincide with fine points;
* explicit schedules (any decreasing orders ending at 1, e.g. 5 -> 4 -> 3
  -> 2 -> 1 as in the paper's by-one schedule) use the same rules;
  with the modal basis the coarse local mode (a, b, c) is the fine local
  mode (a, b, c), a, b, c <= q (Algorithm 2 as printed, for any q < p);
* constrained fine nodes have empty rows of P; coarse levels contain free
  nodes only, so a kept node that is constrained is marked -1 in l2g_next;
* interpolation entries with |value| <= 1e-12 in the 1-D factor are
  structural zeros; duplicates keep their first occurrence (lowest element).
"""
import numpy as np

from .basis import gll_points, lagrange_eval
from .assembly import local_index, csr_from_sorted_or_not

ZERO_TOL = 1e-12


def smallest_prime_factor(p: int) -> int:
    d = 2
    while d * d <= p:
        if p % d == 0:
            return d
        d += 1
    return p


def p_schedule(p: int, schedule=None):
    """Orders visited by p-coarsening, finest first, ending at 1: the given
    coarse orders, or q = p / spf(p) repeatedly."""
    if schedule:
        out = [p] + [int(q) for q in schedule]
        if any(b >= a for a, b in zip(out, out[1:])) or out[-1] < 1:
            raise ValueError("schedule must decrease from p")
        return out
    out = [p]
    while out[-1] > 1:
        out.append(out[-1] // smallest_prime_factor(out[-1]))
    return out


def kept_position(p: int, q: int, a: int) -> int:
    """Fine lattice position (0..p) that numbers coarse nodal position a."""
    return (2 * a * p + q) // (2 * q)


def interp_1d(p: int, q: int, basis: str = "nodal") -> np.ndarray:
    """I1[i, a] = l^q_a(xi^p_i): order-q GLL Lagrange basis at order-p GLL
    points, with |I1| <= 1e-12 set to exact zero.  Modal: the injection
    I1[a, a] = 1 for a <= q (the order-q modes are fine modes)."""
    if basis == "modal":
        I1 = np.zeros((p + 1, q + 1))
        I1[np.arange(q + 1), np.arange(q + 1)] = 1.0
        return I1
    xp, _ = gll_points(p)
    xq, _ = gll_points(q)
    I1 = lagrange_eval(xq, xp).T          # [p+1, q+1]
    I1[np.abs(I1) <= ZERO_TOL] = 0.0
    return I1


def extract_next_dof(p: int, q: int, basis: str = "nodal") -> np.ndarray:
    """Fine local index of each coarse local node, in coarse local order
    (Algorithm 2: modal as printed, nodal reading for GLL nodes)."""
    pos = [kept_position(p, q, a) if basis == "nodal" else a for a in range(q + 1)]
    out = []
    for a in range(q + 1):
        for b in range(q + 1):
            for c in range(q + 1):
                out.append(local_index(p, pos[a], pos[b], pos[c]))
    return np.array(out, dtype=np.int64)


def dof_next(l2g: np.ndarray, p: int, q: int, free: np.ndarray, basis: str = "nodal") -> np.ndarray:
    """Sorted unique fine ids of kept, free nodes (Algorithm 3)."""
    kept = l2g[:, extract_next_dof(p, q, basis)].ravel()
    kept = kept[kept >= 0]
    kept = kept[free[kept]]
    return np.unique(kept)


def l2g_next(l2g: np.ndarray, p: int, q: int, collect: np.ndarray,
             free: np.ndarray, basis: str = "nodal") -> np.ndarray:
    """Coarse ids through the rank in ``collect`` (Algorithm 4); -1 for kept
    nodes that are constrained."""
    kept = l2g[:, extract_next_dof(p, q, basis)].astype(np.int64)
    out = np.full(kept.shape, -1, dtype=np.int64)
    ok = kept >= 0
    ok[ok] = free[kept[ok]]
    out[ok] = np.searchsorted(collect, kept[ok])
    assert np.all(collect[out[ok]] == kept[ok])
    return out.astype(np.int32)


def prolongation(l2g, l2g_nx, p, q, n_fine, n_coarse, free, basis="nodal"):
    """P as COO over elements, sorted by (row, col), first occurrence kept
    (Algorithm 7: injected ones for modal, interpolated values for nodal)."""
    I1 = interp_1d(p, q, basis)
    rows, cols, vals, elems = [], [], [], []
    eidx = np.arange(l2g.shape[0], dtype=np.int64)
    for i in range(p + 1):
        for j in range(p + 1):
            for k in range(p + 1):
                gf = l2g[:, local_index(p, i, j, k)].astype(np.int64)
                fine_ok = gf >= 0
                fine_ok[fine_ok] = free[gf[fine_ok]]
                for a in range(q + 1):
                    for b in range(q + 1):
                        for c in range(q + 1):
                            v = I1[i, a] * I1[j, b] * I1[k, c]
                            if I1[i, a] == 0.0 or I1[j, b] == 0.0 or I1[k, c] == 0.0:
                                continue
                            gc = l2g_nx[:, local_index(q, a, b, c)].astype(np.int64)
                            ok = fine_ok & (gc >= 0)
                            rows.append(gf[ok])
                            cols.append(gc[ok])
                            elems.append(eidx[ok])
                            vals.append(np.full(int(ok.sum()), v))
    r = np.concatenate(rows) if rows else np.zeros(0, dtype=np.int64)
    c = np.concatenate(cols) if cols else np.zeros(0, dtype=np.int64)
    el = np.concatenate(elems) if elems else np.zeros(0, dtype=np.int64)
    v = np.concatenate(vals) if vals else np.zeros(0)
    if n_coarse == 0:
        return csr_from_sorted_or_not(r[:0], c[:0], v[:0], n_fine, 0)
    key = r * n_coarse + c
    order = np.lexsort((el, key))
    key, v = key[order], v[order]
    first = np.ones(key.size, dtype=bool)
    first[1:] = key[1:] != key[:-1]
    # duplicates describe the same basis function at the same node
    grp = np.cumsum(first) - 1
    if key.size:
        ref = v[first][grp]
        assert np.max(np.abs(v - ref)) <= 1e-14
    key, v = key[first], v[first]
    return csr_from_sorted_or_not(key // n_coarse, key % n_coarse, v,
                                  n_fine, n_coarse)


def p_level(l2g, p, q, n_fine, free, basis="nodal"):
    """One p-coarsening step.  Returns (collect, l2g_next, P)."""
    collect = dof_next(l2g, p, q, free, basis)
    l2g_nx = l2g_next(l2g, p, q, collect, free, basis)
    P = prolongation(l2g, l2g_nx, p, q, n_fine, collect.size, free, basis)
    return collect, l2g_nx, P
