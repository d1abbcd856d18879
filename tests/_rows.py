"""Sampled rows of an assembled operator, computed by the oracle from the few
elements around each node (full-size parity where the oracle cannot
assemble the whole operator quickly).  Test infrastructure."""
import numpy as np

from oracle import assembly


def oracle_rows(coords, l2g, p, lam, cons, rows, nq, basis="nodal"):
    """{row: {col: value}} for free rows, constrained columns removed."""
    out = {}
    for r in rows:
        els = np.nonzero((l2g == r).any(axis=1))[0]
        sub = l2g[els]
        acc = {}
        for eids, Ae in assembly.element_matrices(coords, sub, p, nq, lam, basis):
            for e_local, A in zip(eids, Ae):
                g = sub[e_local]
                a = int(np.nonzero(g == r)[0][0])
                for b, c in enumerate(g):
                    if not cons[c]:
                        acc[int(c)] = acc.get(int(c), 0.0) + A[a, b]
        out[r] = acc
    return out
