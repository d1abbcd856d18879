"""The benchmark's 16^3, p = 4 workload (274,625 dofs, 49.5 M nonzeros,
lambda = 10, perturbed vertices seed 2, right-hand side seed 12) against the
whole oracle: the oracle builds this hierarchy in about ten seconds, so here
nothing is sampled.

* every level's CSR structure of A, P and R bit-exact, values within 1e-12
  of the largest entry; every next-level element map and the aggregates;
* FP64 GIAMG-PCG to 1e-10: iterations within +-1, ||x - x_o|| <= 1e-9 ||x_o||;
* a fixed number of iterations (tol = 0): after each iteration j the
  recursive relative residual within 1e-6 of the oracle's (its history), and
  the final iterate within 1e-9;
* the mixed-precision solve (FP32 V-cycle in FP64 flexible CG) within 1e-8
  of the FP64 oracle solution.
"""
import numpy as np
import pytest

import synth
from oracle import hierarchy, krylov

pytestmark = pytest.mark.gpu

N_EL, P_ORD, LAM = 16, 4, 10.0


@pytest.fixture(scope="module")
def full():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2512_15121_amd import giamg
    giamg.library()
    m = synth.hex_mesh(N_EL, P_ORD, perturb=0.1, seed=2)
    H = hierarchy.build(m.coords, m.l2g, P_ORD, LAM, hierarchy.Options())
    b = synth.normal_rhs(m.n_nodes, 12)
    ref = krylov.giamg_pcg(H, b, tol=1e-10)
    assert ref.converged
    return torch, m, H, b, ref


def _solver(m, **kw):
    from paper_2512_15121_amd import Solver, Options
    return Solver(m.coords, m.l2g, P_ORD, LAM, Options(**kw))


def test_whole_hierarchy_against_oracle(full):
    torch, m, H, b, ref = full
    s = _solver(m)
    assert s.num_levels() == len(H.levels)
    assert np.array_equal(s.constrained(), H.constrained)
    for l, lv in enumerate(H.levels):
        rp, ci, val = s.level_csr(l, "A")
        assert np.array_equal(rp, lv.A.indptr) and np.array_equal(ci, lv.A.indices), f"A{l}"
        assert np.max(np.abs(val - lv.A.data)) <= 1e-12 * np.max(np.abs(lv.A.data)), f"A{l}"
        if l + 1 < len(H.levels):
            for which, M in (("P", lv.P), ("R", lv.R)):
                rp, ci, val = s.level_csr(l, which)
                assert np.array_equal(rp, M.indptr) and np.array_equal(ci, M.indices), f"{which}{l}"
                assert np.max(np.abs(val - M.data)) <= 1e-12 * np.max(np.abs(M.data)), f"{which}{l}"
            if lv.agg is not None:
                assert np.array_equal(s.level_aggregates(l), lv.agg)
        if lv.l2g is not None and l > 0:
            assert np.array_equal(s.level_l2g(l), lv.l2g)
    s.close()


def test_fp64_solve_and_residual_history(full):
    torch, m, H, b, ref = full
    s = _solver(m)
    bt = torch.from_numpy(b).to("cuda:0")
    x, info = s.solve(bt, tol=1e-10)
    assert info.status == 0 and abs(info.iters - ref.iters) <= 1
    xh = x.cpu().numpy()
    assert np.linalg.norm(xh - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    s.close()
    k = min(info.iters, ref.iters)
    ref_k = krylov.giamg_pcg(H, b, tol=0.0, maxit=k)
    for j in range(1, k + 1):
        sj = _solver(m, maxit=j)
        xj, ij = sj.solve(bt, tol=0.0)
        assert ij.iters == j
        assert abs(ij.relres - ref_k.history[j]) <= 1e-6 * ref_k.history[j], (j, ij.relres,
                                                                              ref_k.history[j])
        if j == k:
            assert np.linalg.norm(xj.cpu().numpy() - ref_k.x) <= 1e-9 * np.linalg.norm(ref_k.x)
        sj.close()


def test_mixed_solve_against_fp64_oracle(full):
    torch, m, H, b, ref = full
    s = _solver(m, precision="mixed")
    x, info = s.solve(torch.from_numpy(b).to("cuda:0"), tol=1e-10)
    assert info.status == 0 and info.true_relres < 2e-10
    err = np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x)
    assert err <= 1e-8, err
    s.close()
