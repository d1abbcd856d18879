"""Seeded right-hand sides and problem parameters.

All draws use numpy's PCG64 bit generator with an explicit seed so that the
oracle, the tests and the benchmark see identical inputs.
"""
import numpy as np


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def normal_rhs(n_nodes: int, seed) -> np.ndarray:
    """i.i.d. N(0, 1) entries over every node (float64)."""
    return _rng(seed).standard_normal(n_nodes)


def pinned_normal_batch(n_nodes: int, k: int, seed, pin: int = 0) -> np.ndarray:
    """k right-hand sides, row-major [n_nodes, k]: i.i.d. N(0, 1), each
    column shifted to mean zero over all nodes, then the pinned node's entry
    set to zero (pure-Neumann problems with one constrained node)."""
    b = _rng(seed).standard_normal((n_nodes, k))
    b -= b.mean(axis=0, keepdims=True)
    b[pin, :] = 0.0
    return np.ascontiguousarray(b)


def loguniform_lambda(seed, lo: float = 0.1, hi: float = 100.0) -> float:
    """One draw of lambda, log-uniform on [lo, hi]."""
    u = _rng(seed).uniform(np.log(lo), np.log(hi))
    return float(np.exp(u))
