"""Pins of the oracle's smoothers, V-cycle and Krylov loops.

* Chebyshev: on a matrix whose D^-1 A has known eigenpairs, one application
  from zero scales every eigencomponent of the error by
  T_k((b+a-2 mu)/(b-a)) / T_k((b+a)/(b-a));
* weighted Jacobi: the same with (1 - omega mu)^nu;
* power iteration close to the dense largest eigenvalue of D^-1 A;
* the V-cycle operator is symmetric positive definite (dense, tiny problem);
* PCG: against a dense solve; with B = I the textbook CG bound (<= N
  iterations); with B = A^-1 a single iteration; the flexible variant equals
  standard PCG for a fixed SPD preconditioner.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import smoothers, hierarchy, cycle, krylov


def _tridiag(n):
    # D^-1 A = A/2 with eigenvalues 1 - cos(j pi / (n+1)) and sine eigenvectors
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    j = np.arange(1, n + 1)
    mu = 1 - np.cos(j * np.pi / (n + 1))
    V = np.sin(np.outer(np.arange(1, n + 1), j) * np.pi / (n + 1))
    return A, mu, V


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_chebyshev_polynomial(k):
    n = 30
    A, mu, V = _tridiag(n)
    lo, hi = 0.3, 2.1
    dinv = smoothers.diag_inverse(A)
    for col in (0, 7, 15, 29):
        e0 = V[:, col]
        f = A @ e0
        x = smoothers.chebyshev(A, dinv, f, None, k, lo, hi)
        # x0 = 0: error after = e0 - x, i.e. the residual polynomial at mu
        t = (hi + lo - 2 * mu[col]) / (hi - lo)
        s = (hi + lo) / (hi - lo)
        factor = np.cos(k * np.arccos(t)) if abs(t) <= 1 else np.cosh(k * np.arccosh(abs(t))) * np.sign(t) ** k
        factor /= np.cosh(k * np.arccosh(s))
        np.testing.assert_allclose(e0 - x, factor * e0, atol=1e-12)
        # from a nonzero start the error is scaled by the same factor
        x1 = smoothers.chebyshev(A, dinv, f, 0.5 * e0, k, lo, hi)
        np.testing.assert_allclose(e0 - x1, 0.5 * factor * e0, atol=1e-12)


@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_jacobi_polynomial(sweeps):
    A, mu, V = _tridiag(20)
    dinv = smoothers.diag_inverse(A)
    w = 2 / 3
    for col in (0, 9, 19):
        e0 = V[:, col]
        x = smoothers.jacobi(A, dinv, A @ e0, None, sweeps, w)
        np.testing.assert_allclose(e0 - x, (1 - w * mu[col]) ** sweeps * e0, atol=1e-12)


def test_power_iteration_estimate():
    m = synth.hex_mesh(3, 3, perturb=0.1, seed=1)
    H = hierarchy.build(m.coords, m.l2g, 3, 1.0)
    lv = H.levels[0]
    lam = np.max(np.real(np.linalg.eigvals(np.diag(lv.dinv) @ lv.A.toarray())))
    assert 0.9 * lam <= lv.lam_hat <= 1.05 * lam
    v = smoothers.power_start(1000)
    assert np.all(np.abs(v) <= 1) and abs(v.mean()) < 0.1


def _dense_B(H):
    n = H.levels[0].A.shape[0]
    B = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1
        B[:, i] = cycle.vcycle(H, e)
    return B


@pytest.mark.parametrize("smoother,deg", [("chebyshev", 2), ("jacobi", 2), ("chebyshev", 3)])
def test_vcycle_spd(smoother, deg):
    m = synth.hex_mesh(2, 4, perturb=0.1, seed=3)
    H = hierarchy.build(m.coords, m.l2g, 4, 1.0,
                        hierarchy.Options(smoother=smoother, degree=deg))
    B = _dense_B(H)
    assert np.max(np.abs(B - B.T)) <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    # as a stationary iteration the V-cycle contracts the error
    A = H.levels[0].A.toarray()
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(A.shape[0]) - B @ A)))
    assert rho < 1


def test_coarsest_cholesky_solve():
    m = synth.hex_mesh(4, 1, perturb=0.1, seed=3)
    H = hierarchy.build(m.coords, m.l2g, 1, 1.0)
    lv = H.levels[-1]
    f = np.arange(lv.A.shape[0], dtype=float)
    np.testing.assert_allclose(cycle.coarse_solve(lv, f),
                               np.linalg.solve(lv.A.toarray(), f), rtol=1e-12)


def test_pcg_against_dense_and_textbook():
    m = synth.hex_mesh(3, 2, perturb=0.1, seed=9)
    H = hierarchy.build(m.coords, m.l2g, 2, 1.0)
    A = H.levels[0].A
    b = synth.normal_rhs(m.n_nodes, 4)
    res = krylov.giamg_pcg(H, b, tol=1e-12)
    x = np.linalg.solve(A.toarray(), b)
    assert res.converged and np.linalg.norm(res.x - x) <= 1e-10 * np.linalg.norm(x)
    assert res.true_relres < 1e-11
    # B = I: plain CG terminates within N steps
    r0 = krylov.pcg(A, b, lambda r: r.copy(), tol=1e-10, maxit=2000)
    assert r0.converged and r0.iters <= A.shape[0]
    # B = A^-1: one step
    Ainv = np.linalg.inv(A.toarray())
    r1 = krylov.pcg(A, b, lambda r: Ainv @ r, tol=1e-10)
    assert r1.iters == 1
    # the flexible beta equals the standard one for a fixed SPD B
    rf = krylov.giamg_pcg(H, b, tol=1e-10, flexible=True)
    rs = krylov.giamg_pcg(H, b, tol=1e-10)
    assert abs(rf.iters - rs.iters) <= 1
    np.testing.assert_allclose(rf.history[:rs.iters], rs.history[:rs.iters], rtol=1e-6)
    # zero right-hand side and a converged initial guess
    assert krylov.giamg_pcg(H, np.zeros_like(b)).iters == 0
    assert krylov.giamg_pcg(H, b, x0=x).iters == 0


def test_manufactured_4cube_converges_order_robust():
    iters = []
    for p in (2, 3, 4):
        m = synth.hex_mesh(4, p)
        H = hierarchy.build(m.coords, m.l2g, p, 1.0)
        res = krylov.giamg_pcg(H, synth.normal_rhs(m.n_nodes, 1))
        assert res.converged and res.true_relres < 1e-9
        iters.append(res.iters)
    assert max(iters) <= 2 * min(iters) + 5


def test_jacobi_pcg_exact_on_a_diagonal_matrix():
    """With A diagonal the preconditioner is A^-1: one iteration solves."""
    import scipy.sparse as sp
    d = np.linspace(0.5, 40.0, 30)
    b = np.sin(np.arange(30.0))
    res = krylov.jacobi_pcg(sp.diags(d).tocsr(), b, tol=1e-14)
    assert res.iters == 1 and np.allclose(res.x, b / d, rtol=1e-15, atol=0)


def test_jacobi_pcg_is_cg_on_the_scaled_system():
    """Jacobi-PCG on A x = b produces x_k = D^-1/2 y_k, y_k the iterates of
    plain CG on (D^-1/2 A D^-1/2) y = D^-1/2 b (the classical equivalence),
    written here as a textbook CG loop on the scaled matrix."""
    import scipy.sparse as sp
    import synth
    from oracle import assembly
    m = synth.hex_mesh(3, 3, perturb=0.15, seed=8)
    A, _ = assembly.assemble(m.coords, m.l2g, 3, 2.0)
    b = synth.normal_rhs(m.n_nodes, 3)
    s = 1.0 / np.sqrt(A.diagonal())
    S = sp.diags(s)
    Ah = (S @ A @ S).tocsr()
    bh = s * b
    for k in (1, 5, 17):
        y = np.zeros_like(bh)
        r = bh.copy()
        pdir = r.copy()
        rr = r @ r
        for _ in range(k):
            q = Ah @ pdir
            alpha = rr / (pdir @ q)
            y += alpha * pdir
            r -= alpha * q
            rr_new = r @ r
            pdir = r + (rr_new / rr) * pdir
            rr = rr_new
        res = krylov.jacobi_pcg(A, b, tol=0.0, maxit=k)
        assert res.iters == k
        assert np.linalg.norm(res.x - s * y) <= 1e-11 * np.linalg.norm(s * y)
    full = krylov.jacobi_pcg(A, b, tol=1e-12)
    ref = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(full.x - ref) <= 1e-9 * np.linalg.norm(ref)
