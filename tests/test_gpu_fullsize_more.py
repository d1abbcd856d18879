"""Full-size parity at the two other benchmark workloads, in the launch
configurations bench.py times, on outputs the oracle computes one by one:

* 32^3 hexahedra, p = 4 (2,146,689 dofs, 423.7 M nonzeros), lambda
  log-uniform (seed 13): every p-level element map bit-exact, sampled fine
  rows, an FP64 solve checked on sampled residual rows, and the mixed
  (FP32 V-cycle, FP64 flexible CG) solve within 1e-8 of it;
* 20^3 hexahedra, p = 3, pure Neumann with node 0 pinned, 64 right-hand
  sides (mixed, block products, graph replay): sampled residual rows of
  every column, and columns bit-identical to the same right-hand side
  solved alone.
"""
import numpy as np
import pytest

import synth
from _rows import oracle_rows
from oracle import assembly, ptransfer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def test_helmholtz32_p4_fullsize(torch_mod):
    torch = torch_mod
    from paper_2512_15121_amd import Solver, Options
    n, p = 32, 4
    lam = synth.loguniform_lambda(13)
    m = synth.hex_mesh(n, p, perturb=0.1, seed=3)
    cons = assembly.boundary_nodes(m.l2g, p, m.n_nodes)
    s = Solver(m.coords, m.l2g, p, lam, Options())
    assert np.array_equal(s.constrained(), cons)
    # integer work: every p-level's element map
    l2g, free = m.l2g, ~cons
    for lvl, (pf, q) in enumerate(zip(ptransfer.p_schedule(p)[:-1], ptransfer.p_schedule(p)[1:]),
                                  start=1):
        collect = ptransfer.dof_next(l2g, pf, q, free)
        nxt = ptransfer.l2g_next(l2g, pf, q, collect, free)
        assert np.array_equal(s.level_l2g(lvl), nxt)
        l2g, free = nxt, np.ones(collect.size, dtype=bool)
    # sampled fine rows
    rng = np.random.default_rng(0)
    rows = rng.choice(np.nonzero(~cons)[0], 20, replace=False)
    ref = oracle_rows(m.coords, m.l2g, p, lam, cons, rows, p + 2)
    rp, ci, val = s.level_csr(0, "A")
    for r in rows:
        cols = ci[rp[r]:rp[r + 1]]
        assert list(cols) == sorted(ref[r])
        rv = np.array([ref[r][c] for c in cols])
        assert np.max(np.abs(val[rp[r]:rp[r + 1]] - rv)) <= 1e-13 * np.max(np.abs(rv))
    del rp, ci, val
    # FP64 solve: residual on sampled rows
    b = synth.normal_rhs(m.n_nodes, 23)
    bt = torch.from_numpy(b).to("cuda:0")
    x, info = s.solve(bt, tol=1e-10)
    assert info.status == 0 and info.true_relres < 2e-10
    xh = x.cpu().numpy()
    bn = np.linalg.norm(b)
    for r in rows:
        res = b[r] - sum(v * xh[c] for c, v in ref[r].items())
        assert abs(res) <= 2e-10 * bn
    s.close()
    # mixed precision on the same problem
    sm = Solver(m.coords, m.l2g, p, lam, Options(precision="mixed"))
    xm, im = sm.solve(bt, tol=1e-10)
    assert im.status == 0 and im.true_relres < 2e-10
    assert np.linalg.norm(xm.cpu().numpy() - xh) <= 1e-8 * np.linalg.norm(xh)
    sm.close()


def test_poisson20_p3_pinned_batch64_fullsize(torch_mod):
    torch = torch_mod
    from paper_2512_15121_amd import Solver, Options
    n, p, k = 20, 3, 64
    m = synth.hex_mesh(n, p, perturb=0.1, seed=4)
    cons = np.zeros(m.n_nodes, dtype=bool)
    cons[0] = True
    B = synth.pinned_normal_batch(m.n_nodes, k, 14)
    s = Solver(m.coords, m.l2g, p, 0.0, Options(bc="pin", precision="mixed"))
    Bt = torch.from_numpy(B).to("cuda:0")
    X, infos = s.solve_batch(Bt, tol=1e-10)
    assert all(i.status == 0 and i.true_relres < 2e-10 for i in infos)
    Xh = X.cpu().numpy()
    rng = np.random.default_rng(1)
    rows = rng.choice(np.arange(1, m.n_nodes), 12, replace=False)
    ref = oracle_rows(m.coords, m.l2g, p, 0.0, cons, rows, p + 2)
    for j in range(k):
        bn = np.linalg.norm(B[:, j])
        for r in rows:
            res = B[r, j] - sum(v * Xh[c, j] for c, v in ref[r].items())
            assert abs(res) <= 2e-10 * bn, (j, r)
    # a column gives the same bits alone and inside the batch
    for j in (0, 37):
        Xj, ij = s.solve_batch(Bt[:, j:j + 1].contiguous(), tol=1e-10)
        assert ij[0].iters == infos[j].iters and torch.equal(Xj[:, 0], X[:, j])
    s.close()
