"""Batched solves (block SpMM V-cycle, per-column CG, graph replay) against
the oracle, and the reproducibility contract: a right-hand side gives the same
bits alone or inside a batch."""
import numpy as np
import pytest

import synth
from oracle import hierarchy, krylov

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2512_15121_amd import giamg
    giamg.library()
    n, p = 5, 3
    m = synth.hex_mesh(n, p, perturb=0.1, seed=4)
    H = hierarchy.build(m.coords, m.l2g, p, 0.0,
                        hierarchy.Options(bc="pin", coarse_max=100))
    return torch, torch.device("cuda:0"), m, H


def _solver(m, precision):
    from paper_2512_15121_amd import Solver, Options
    return Solver(m.coords, m.l2g, 3, 0.0, Options(bc="pin", coarse_max=100, precision=precision))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_against_oracle(env, precision):
    torch, dev, m, H = env
    k = 8
    B = synth.pinned_normal_batch(m.n_nodes, k, 14)
    s = _solver(m, precision)
    X, infos = s.solve_batch(torch.from_numpy(B).to(dev), tol=1e-10)
    Xh = X.cpu().numpy()
    for j in range(k):
        ref = krylov.giamg_pcg(H, B[:, j].copy(), tol=1e-10)
        assert infos[j].status == 0 and infos[j].true_relres < 1e-9
        err = np.linalg.norm(Xh[:, j] - ref.x) / np.linalg.norm(ref.x)
        if precision == "fp64":
            assert abs(infos[j].iters - ref.iters) <= 1
            assert err <= 1e-9, (j, err)
        else:
            assert abs(infos[j].iters - ref.iters) <= 2
            assert err <= 1e-8, (j, err)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_column_alone_is_bitwise_identical(env, precision):
    torch, dev, m, H = env
    k = 6
    B = synth.pinned_normal_batch(m.n_nodes, k, 21)
    s = _solver(m, precision)
    X, infos = s.solve_batch(torch.from_numpy(B).to(dev), tol=1e-10)
    for j in (0, 3, 5):
        Xj, ij = s.solve_batch(torch.from_numpy(B[:, j:j + 1].copy()).to(dev), tol=1e-10)
        assert ij[0].iters == infos[j].iters
        assert torch.equal(Xj[:, 0], X[:, j])
    # a batch that mixes in a zero column and a repeated column
    B2 = np.concatenate([B[:, :2], np.zeros((m.n_nodes, 1)), B[:, :1]], axis=1)
    X2, i2 = s.solve_batch(torch.from_numpy(np.ascontiguousarray(B2)).to(dev), tol=1e-10)
    assert i2[2].iters == 0 and torch.count_nonzero(X2[:, 2]).item() == 0
    assert torch.equal(X2[:, 0], X[:, 0]) and torch.equal(X2[:, 3], X[:, 0])
    assert torch.equal(X2[:, 1], X[:, 1])
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("smoother,degree", [("chebyshev", 1), ("chebyshev", 3), ("chebyshev", 4),
                                             ("jacobi", 3)])
def test_batch_smoother_degrees_against_oracle(env, precision, smoother, degree):
    """The block smoothers at every recurrence length (degree 1: one damped
    step; 3 and 4: middle steps of the three-term recurrence; Jacobi sweeps),
    per column against the oracle's single solve.  The mixed path is flexible
    CG around an FP32 cycle: its bar is the error against the FP64 oracle
    and the true residual; its iteration count may drift a few from the FP64
    count (a quarter, at least two) as the FP32 preconditioner changes the
    Krylov space."""
    torch, dev, m, _ = env
    from paper_2512_15121_amd import Solver, Options
    H = hierarchy.build(m.coords, m.l2g, 3, 0.0,
                        hierarchy.Options(bc="pin", coarse_max=100, smoother=smoother,
                                          degree=degree))
    k = 5
    B = synth.pinned_normal_batch(m.n_nodes, k, 40 + degree)
    s = Solver(m.coords, m.l2g, 3, 0.0, Options(bc="pin", coarse_max=100, precision=precision,
                                                smoother=smoother, degree=degree))
    X, infos = s.solve_batch(torch.from_numpy(B).to(dev), tol=1e-10)
    Xh = X.cpu().numpy()
    for j in range(k):
        ref = krylov.giamg_pcg(H, B[:, j].copy(), tol=1e-10)
        assert infos[j].status == 0 and infos[j].true_relres < 1e-9
        err = np.linalg.norm(Xh[:, j] - ref.x) / np.linalg.norm(ref.x)
        if precision == "fp64":
            assert abs(infos[j].iters - ref.iters) <= 1 and err <= 1e-9, (j, err)
        else:
            assert abs(infos[j].iters - ref.iters) <= max(2, ref.iters // 4), (j, infos[j].iters)
            assert err <= 1e-8, (j, err)
    s.close()


def test_batch_iteration_cap(env):
    torch, dev, m, H = env
    from paper_2512_15121_amd import Solver, Options, giamg
    s = Solver(m.coords, m.l2g, 3, 0.0, Options(bc="pin", coarse_max=100, maxit=2))
    B = synth.pinned_normal_batch(m.n_nodes, 3, 2)
    X, infos = s.solve_batch(torch.from_numpy(B).to(dev), tol=1e-10)
    assert all(i.status == giamg.ENOTCONV and i.iters == 2 for i in infos)
    s.close()


def _shape_solutions(torch, dev, m, p, lam, bc, precision, B):
    from paper_2512_15121_amd import Solver, Options
    out = {}
    for kind in ("lanes", "wave", "group"):
        s = Solver(m.coords, m.l2g, p, lam, Options(bc=bc, coarse_max=100, precision=precision,
                                                    batch_kernel=kind))
        X, infos = s.solve_batch(torch.from_numpy(B).to(dev), tol=1e-10)
        out[kind] = (X, [(i.iters, i.status) for i in infos])
        s.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["p3_pin", "p4_dirichlet"])
def test_batch_kernel_shapes_give_the_same_bits(env, precision, case):
    """Every block-product shape (lanes per row, a row per wavefront, a group
    of rows with one column list per wavefront) sums each row in CSR order, so
    the whole batched solve is bitwise the same.  k = 70: two 64-column tiles,
    the second ragged.  p = 3 groups rows by 8, 4, 2 and 1; p = 4 (27, 9 and 3
    rows per pattern, Dirichlet rows single) by 7, 6, 5, 4, 3 and 1."""
    torch, dev, m, H = env
    k = 70
    if case == "p3_pin":
        p, lam, bc = 3, 0.0, "pin"
        B = synth.pinned_normal_batch(m.n_nodes, k, 33)
    else:
        p, lam, bc = 4, 2.0, "dirichlet"
        m = synth.hex_mesh(3, 4, perturb=0.1, seed=6)
        B = np.ascontiguousarray(synth.normal_rhs(m.n_nodes * k, 34).reshape(m.n_nodes, k))
    out = _shape_solutions(torch, dev, m, p, lam, bc, precision, B)
    X0, it0 = out["lanes"]
    assert all(st == 0 for _, st in it0)
    for kind in ("wave", "group"):
        X, it = out[kind]
        assert it == it0, kind
        assert torch.equal(X, X0), kind
