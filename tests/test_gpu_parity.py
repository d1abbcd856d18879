"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Bars (each from the rounding of the operation it checks):
* integer work bit-exact: constrained mask, every level's CSR structure of
  A, P, R and A P, next-level element maps, aggregates;
* assembled/Galerkin values: max |a - a_o| <= 1e-12 max |a_o| per level
  (for A P: 1e-12 max (|A| |P|), as its entries cancel);
* lambda_max estimate: relative 1e-6;
* one product: |y - y_o|_i <= 64 eps (|A| |x|)_i;
* smoothing, V-cycle, coarsest solve: max_i |y - y_o|_i <= 1e-11 max_i |y_o|_i;
* FP64 solve at 1e-10: CG iterations within +-1, ||x - x_o|| <= 1e-9 ||x_o||;
  with a fixed iteration count (tol = 0) the same bound on x.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import hierarchy, krylov, cycle, smoothers, assembly, galerkin

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2512_15121_amd import giamg
    giamg.library()            # fails loudly if the HIP library is missing
    return torch, torch.device("cuda:0")


CASES = {
    # name: (n, p, lam, smoother, perturb, coarse_max, bc, basis, schedule)
    "manufactured_4cube_p2_jacobi": (4, 2, 1.0, "jacobi", 0.0, 2000, "dirichlet", "nodal", ()),
    "p4_6cube_cheb_sa": (6, 4, 10.0, "chebyshev", 0.1, 100, "dirichlet", "nodal", ()),
    "p6_4cube_cheb": (4, 6, 0.5, "chebyshev", 0.1, 2000, "dirichlet", "nodal", ()),
    "p5_7cube_ragged": (7, 5, 3.0, "chebyshev", 0.1, 300, "dirichlet", "nodal", ()),
    "p3_pin_neumann": (5, 3, 0.0, "chebyshev", 0.1, 100, "pin", "nodal", ()),
    # the appendix's modal basis: injection transfers (Algorithm 7)
    "modal_p4_5cube_sa": (5, 4, 10.0, "chebyshev", 0.1, 100, "dirichlet", "modal", ()),
    "modal_p6_3cube": (3, 6, 1.0, "chebyshev", 0.1, 2000, "dirichlet", "modal", ()),
    "modal_p3_pin_neumann": (4, 3, 0.0, "chebyshev", 0.1, 100, "pin", "modal", ()),
    # the by-one schedule (non-divisor nodal steps: nearest-lattice numbering)
    "p5_5cube_by_one": (5, 5, 2.0, "chebyshev", 0.1, 100, "dirichlet", "nodal", (4, 3, 2, 1)),
    "modal_p5_4cube_by_one": (4, 5, 2.0, "chebyshev", 0.1, 100, "dirichlet", "modal", (4, 3, 2, 1)),
    # Table 1's mesh and order with the boundary nodes kept on the coarse
    # levels (8 -> 4 -> 2 -> 1, coarsest 27 / 343)
    "p8_2cube_keep_boundary": (2, 8, 1.0, "chebyshev", 0.1, 2000, "dirichlet", "nodal", ()),
    # Chebyshev degrees other than 2 (Section 3.2, number of smoothing
    # iterations): degree 1 (a single damped step, no recurrence), 3 and 4
    # (middle steps of the three-term recurrence); weighted Jacobi with 3 sweeps
    "p4_5cube_cheb1_sa": (5, 4, 10.0, "chebyshev", 0.1, 100, "dirichlet", "nodal", ()),
    "p3_6cube_cheb3_sa": (6, 3, 2.0, "chebyshev", 0.1, 100, "dirichlet", "nodal", ()),
    "p6_3cube_cheb4": (3, 6, 0.5, "chebyshev", 0.1, 2000, "dirichlet", "nodal", ()),
    "p4_4cube_jacobi3": (4, 4, 1.0, "jacobi", 0.1, 100, "dirichlet", "nodal", ()),
    # a strength threshold on the aggregation graph (Section 2.5): the
    # order-1 level's weak couplings drop out, 12 aggregates instead of 6
    "p4_6cube_theta": (6, 4, 10.0, "chebyshev", 0.1, 100, "dirichlet", "nodal", ()),
}
# further options per case (oracle and library take the same names); Table
# 1's case runs Chebyshev of degree 3 as the paper's experiment does
CASE_OPTS = {"p8_2cube_keep_boundary": {"keep_boundary": True, "degree": 3},
             "p4_5cube_cheb1_sa": {"degree": 1},
             "p3_6cube_cheb3_sa": {"degree": 3},
             "p6_3cube_cheb4": {"degree": 4},
             "p4_4cube_jacobi3": {"degree": 3},
             "p4_6cube_theta": {"theta": 0.05}}


def _maxnorm_close(got, ref, rel):
    """Max-norm comparison of a whole vector: every entry within rel of the
    largest entry of the reference."""
    return np.max(np.abs(got - ref)) <= rel * np.max(np.abs(ref))

_cache = {}


def _case(name):
    if name not in _cache:
        n, p, lam, sm, pert, cm, bc, basis, sched = CASES[name]
        m = synth.hex_mesh(n, p, perturb=pert, seed=2, basis=basis)
        H = hierarchy.build(m.coords, m.l2g, p, lam,
                            hierarchy.Options(smoother=sm, coarse_max=cm, bc=bc, basis=basis,
                                              schedule=list(sched) or None, **CASE_OPTS.get(name, {})))
        _cache[name] = (m, H)
    return _cache[name]


def _solver(name, precision="fp64", **kw):
    from paper_2512_15121_amd import Solver, Options
    n, p, lam, sm, pert, cm, bc, basis, sched = CASES[name]
    m, _ = _case(name)
    return Solver(m.coords, m.l2g, p, lam,
                  Options(smoother=sm, coarse_max=cm, bc=bc, precision=precision, basis=basis,
                          schedule=tuple(sched), **{**CASE_OPTS.get(name, {}), **kw}))


def _max_row(M):
    return int(np.max(np.diff(M.tocsr().indptr)))


def _to(torch, dev, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


@pytest.mark.parametrize("name", list(CASES))
def test_hierarchy_bitexact_structure_and_values(torch_dev, name):
    m, H = _case(name)
    s = _solver(name)
    assert s.num_levels() == len(H.levels)
    assert np.array_equal(s.constrained(), H.constrained)
    for l, lv in enumerate(H.levels):
        d = s.level(l)
        assert d["rows"] == lv.A.shape[0]
        is_h = l > 0 and H.levels[l - 1].agg is not None
        assert d["kind"] == ("h" if is_h else "p") and d["order"] == lv.order
        rp, ci, val = s.level_csr(l, "A")
        assert np.array_equal(rp, lv.A.indptr) and np.array_equal(ci, lv.A.indices), f"A{l}"
        assert np.max(np.abs(val - lv.A.data)) <= 1e-12 * np.max(np.abs(lv.A.data)), f"A{l}"
        if l + 1 < len(H.levels):
            for which, M in (("P", lv.P), ("R", lv.R)):
                rp, ci, val = s.level_csr(l, which)
                assert np.array_equal(rp, M.indptr) and np.array_equal(ci, M.indices), f"{which}{l}"
                assert np.max(np.abs(val - M.data)) <= 1e-12 * np.max(np.abs(M.data)), f"{which}{l}"
            # A P, the left factor of the Galerkin product, kept for post-smoothing
            AP = galerkin.values_on_pattern(galerkin.symbolic_product(lv.A, lv.P), lv.A @ lv.P)
            rp, ci, val = s.level_csr(l, "AP")
            assert d["nnz_AP"] == AP.nnz
            assert np.array_equal(rp, AP.indptr) and np.array_equal(ci, AP.indices), f"AP{l}"
            scale = (abs(lv.A) @ abs(lv.P)).max()
            assert np.max(np.abs(val - AP.data)) <= 1e-12 * scale, f"AP{l}"
            assert abs(d["lam_hat"] - lv.lam_hat) <= 1e-6 * lv.lam_hat
            if lv.agg is not None:
                assert np.array_equal(s.level_aggregates(l), lv.agg)
        if lv.l2g is not None and l > 0:
            assert np.array_equal(s.level_l2g(l), lv.l2g)
    s.close()


def test_table1_hierarchy_on_device(torch_dev):
    """Table 1's mesh and order with keep_boundary: the device hierarchy has
    the printed 4 levels and a coarsest level of 27 rows / 343 nonzeros."""
    s = _solver("p8_2cube_keep_boundary")
    d = [s.level(l) for l in range(s.num_levels())]
    assert [(x["order"], x["rows"]) for x in d] == [(8, 17 ** 3), (4, 9 ** 3), (2, 5 ** 3), (1, 27)]
    assert d[-1]["coarsest"] and d[-1]["nnz_A"] == 343
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_staged_gathers_bitwise_equal_direct(torch_dev, name):
    """Products with each row block's columns staged in LDS multiply the same
    operands and sum in the same order as direct gathers: every operator
    product, the V-cycle and the whole solve agree bit for bit."""
    torch, dev = torch_dev
    s1 = _solver(name, lean_max_nnz=0)
    s2 = _solver(name, direct_gathers=True, lean_max_nnz=0)
    d0 = s1.level(0)
    assert d0["groups_A"] == 0 and not d0["lean_A"]
    assert d0["staged_nnz_A"] > 0.9 * d0["nnz_A"] and d0["runs_A"] > 0
    assert s2.level(0)["staged_nnz_A"] == 0 and s2.level(0)["runs_A"] == 0
    rng = np.random.default_rng(7)
    nl = s1.num_levels()
    for l in range(nl):
        n = s1.level(l)["rows"]
        x = _to(torch, dev, rng.standard_normal(n))
        o1 = torch.zeros(n, dtype=torch.float64, device=dev)
        o2 = torch.zeros_like(o1)
        s1.apply("spmv", l, x, out=o1)
        s2.apply("spmv", l, x, out=o2)
        assert torch.equal(o1, o2), f"spmv {l}"
        if l + 1 == nl:
            continue
        nc = s1.level(l + 1)["rows"]
        c1 = torch.zeros(nc, dtype=torch.float64, device=dev)
        c2 = torch.zeros_like(c1)
        s1.apply("restrict", l, x, out=c1)
        s2.apply("restrict", l, x, out=c2)
        assert torch.equal(c1, c2), f"restrict {l}"
        y1, y2 = x.clone(), x.clone()
        s1.apply("prolong_add", l, c1, out=y1)
        s2.apply("prolong_add", l, c1, out=y2)
        assert torch.equal(y1, y2), f"prolong {l}"
        s1.apply("vcycle", l, x, out=o1)
        s2.apply("vcycle", l, x, out=o2)
        assert torch.equal(o1, o2), f"vcycle {l}"
    b = _to(torch, dev, rng.standard_normal(d0["rows"]))
    x1, i1 = s1.solve(b, tol=1e-10)
    x2, i2 = s2.solve(b, tol=1e-10)
    assert i1.iters == i2.iters and i1.relres == i2.relres and torch.equal(x1, x2)
    s1.close()
    s2.close()


def test_staged_gathers_mixed_bitwise_equal_direct(torch_dev):
    torch, dev = torch_dev
    name = "p4_6cube_cheb_sa"
    s1 = _solver(name, precision="mixed", lean_max_nnz=0)
    s2 = _solver(name, precision="mixed", direct_gathers=True, lean_max_nnz=0)
    b = _to(torch, dev, np.random.default_rng(8).standard_normal(s1.level(0)["rows"]))
    x1, i1 = s1.solve(b, tol=1e-10)
    x2, i2 = s2.solve(b, tol=1e-10)
    assert i1.status == 0 and i1.iters == i2.iters and torch.equal(x1, x2)
    s1.close()
    s2.close()


def _levels_bitwise(torch, dev, s1, s2, fp32=False):
    """spmv, restriction, prolongation and the V-cycle of every level agree
    bit for bit between two solvers of the same hierarchy."""
    rng = np.random.default_rng(11)
    dt = torch.float32 if fp32 else torch.float64
    nl = s1.num_levels()
    for l in range(nl):
        n = s1.level(l)["rows"]
        x = _to(torch, dev, rng.standard_normal(n), dt)
        o1 = torch.zeros(n, dtype=dt, device=dev)
        o2 = torch.zeros_like(o1)
        s1.apply("spmv", l, x, out=o1, fp32=fp32)
        s2.apply("spmv", l, x, out=o2, fp32=fp32)
        assert torch.equal(o1, o2), f"spmv {l}"
        if l + 1 == nl:
            continue
        nc = s1.level(l + 1)["rows"]
        c1 = torch.zeros(nc, dtype=dt, device=dev)
        c2 = torch.zeros_like(c1)
        s1.apply("restrict", l, x, out=c1, fp32=fp32)
        s2.apply("restrict", l, x, out=c2, fp32=fp32)
        assert torch.equal(c1, c2), f"restrict {l}"
        y1, y2 = x.clone(), x.clone()
        s1.apply("prolong_add", l, c1, out=y1, fp32=fp32)
        s2.apply("prolong_add", l, c1, out=y2, fp32=fp32)
        assert torch.equal(y1, y2), f"prolong {l}"
        s1.apply("vcycle", l, x, out=o1, fp32=fp32)
        s2.apply("vcycle", l, x, out=o2, fp32=fp32)
        assert torch.equal(o1, o2), f"vcycle {l}"


@pytest.mark.parametrize("name", list(CASES))
def test_grouped_form_rows_bitwise_equal_csr(torch_dev, name):
    """The grouped form (rows with one column list share their slots, values
    in per-block planes) sums every row in the CSR form's order: products,
    transfers and V-cycles of every level agree bit for bit.  A solve differs
    only through the CG dot products, whose block partials add the rows in
    another order: same iterations, iterates equal to rounding."""
    torch, dev = torch_dev
    n, p, lam, sm, pert, cm, bc, basis, sched = CASES[name]
    s1 = _solver(name, row_groups=True, lean_max_nnz=0)
    s2 = _solver(name, lean_max_nnz=0)
    d1, d2 = s1.level(0), s2.level(0)
    assert d2["groups_A"] == 0 and d2["group_entries_A"] == 0
    if p >= 3 and _max_row(_case(name)[1].levels[0].A) <= 4096:
        # interior, face and edge nodes share column lists (longer rows: CSR form)
        assert d1["groups_A"] > 0 and d1["group_entries_A"] <= 0.8 * d1["nnz_A"]
        assert d1["staged_nnz_A"] == 0 and d1["runs_A"] == 0
    _levels_bitwise(torch, dev, s1, s2)
    b = _to(torch, dev, np.random.default_rng(12).standard_normal(d1["rows"]))
    x1, i1 = s1.solve(b, tol=1e-10)
    x2, i2 = s2.solve(b, tol=1e-10)
    assert i1.status == 0 and i2.status == 0 and abs(i1.iters - i2.iters) <= 1
    assert torch.linalg.norm(x1 - x2) <= 1e-10 * torch.linalg.norm(x2)
    s1.close()
    s2.close()


@pytest.mark.parametrize("name", list(CASES))
def test_lean_form_rows_bitwise_equal_csr(torch_dev, name):
    """Operators up to lean_max_nnz nonzeros run the row-direct kernel: every
    level's products, transfers and V-cycle equal the CSR form's bit for bit
    (FP64, and FP32 for the mixed hierarchy); solves agree to rounding (the
    CG dot partials of a lean fine level add rows over other blocks)."""
    torch, dev = torch_dev
    s1 = _solver(name, lean_max_nnz=10 ** 9)   # every operator lean (rows up to 8192)
    s2 = _solver(name, lean_max_nnz=0)
    fits = _max_row(_case(name)[1].levels[0].A) <= 8192
    assert s1.level(0)["lean_A"] == fits and not s2.level(0)["lean_A"]
    if fits:
        assert s1.level(0)["staged_nnz_A"] == 0 and s1.level(0)["runs_A"] == 0
    _levels_bitwise(torch, dev, s1, s2)
    b = _to(torch, dev, np.random.default_rng(14).standard_normal(s1.level(0)["rows"]))
    x1, i1 = s1.solve(b, tol=1e-10)
    x2, i2 = s2.solve(b, tol=1e-10)
    assert i1.status == 0 and i2.status == 0 and abs(i1.iters - i2.iters) <= 1
    assert torch.linalg.norm(x1 - x2) <= 1e-10 * torch.linalg.norm(x2)
    s1.close()
    s2.close()
    m1 = _solver(name, precision="mixed", lean_max_nnz=10 ** 9)
    m2 = _solver(name, precision="mixed", lean_max_nnz=0)
    _levels_bitwise(torch, dev, m1, m2, fp32=True)
    m1.close()
    m2.close()


def test_lean_threshold_picks_small_operators(torch_dev):
    """The default threshold leaves the fine operator of a mid-size case in
    the staged CSR form and moves the small coarse levels to the lean form."""
    name = "p4_6cube_cheb_sa"
    s = _solver(name)
    levels = [s.level(l) for l in range(s.num_levels())]
    for d in levels:
        assert d["lean_A"] == (d["nnz_A"] <= 2000000)
    assert not levels[0]["lean_A"] and levels[0]["staged_nnz_A"] > 0
    assert any(d["lean_A"] for d in levels[1:])
    s.close()


@pytest.mark.parametrize("name", ["p4_6cube_cheb_sa", "modal_p5_4cube_by_one"])
def test_grouped_form_fp32_rows_bitwise_equal_csr(torch_dev, name):
    torch, dev = torch_dev
    s1 = _solver(name, precision="mixed", row_groups=True, lean_max_nnz=0)
    s2 = _solver(name, precision="mixed", lean_max_nnz=0)
    assert s1.level(0)["groups_A"] > 0
    _levels_bitwise(torch, dev, s1, s2, fp32=True)
    b = _to(torch, dev, np.random.default_rng(13).standard_normal(s1.level(0)["rows"]))
    x1, i1 = s1.solve(b, tol=1e-10)
    x2, i2 = s2.solve(b, tol=1e-10)
    assert i1.status == 0 and i2.status == 0 and abs(i1.iters - i2.iters) <= 1
    assert torch.linalg.norm(x1 - x2) <= 1e-9 * torch.linalg.norm(x2)
    s1.close()
    s2.close()


@pytest.mark.parametrize("name", ["modal_p4_5cube_sa", "modal_p6_3cube", "modal_p3_pin_neumann"])
def test_modal_galerkin_is_principal_submatrix_on_device(torch_dev, name):
    """With injection P the device Galerkin product R (A P) sums one term per
    entry: each coarse p-level operator is the finer one restricted to the
    kept modes, bit for bit (and P holds ones only)."""
    m, H = _case(name)
    s = _solver(name)
    for l, lv in enumerate(H.levels[:-1]):
        if lv.collect is None:
            break
        rp, ci, val = s.level_csr(l, "A")
        A = sp.csr_matrix((val, ci, rp), shape=(rp.size - 1, rp.size - 1))
        prp, pci, pval = s.level_csr(l, "P")
        assert np.all(pval == 1.0) and np.array_equal(pci, lv.P.indices)
        rc, cc, vc = s.level_csr(l + 1, "A")
        Ac = sp.csr_matrix((vc, cc, rc), shape=(rc.size - 1, rc.size - 1))
        sub = A[lv.collect][:, lv.collect]
        assert abs(sub - Ac).max() == 0.0, f"level {l}"
    s.close()


@pytest.mark.parametrize("name", ["p4_6cube_cheb_sa", "p3_pin_neumann", "manufactured_4cube_p2_jacobi",
                                  "modal_p4_5cube_sa", "p4_5cube_cheb1_sa", "p3_6cube_cheb3_sa",
                                  "p6_3cube_cheb4", "p4_4cube_jacobi3", "p8_2cube_keep_boundary",
                                  "p4_6cube_theta"])
def test_each_vcycle_step(torch_dev, name):
    """Each step of the V-cycle on one level.  Products, residuals and
    transfers are held to the rounding bound of the product on the operator
    the kernel multiplies -- the device's own CSR values, which equal the
    oracle's to 1e-12 of the largest entry (test_hierarchy_bitexact_...);
    against the oracle's operator the entries of high-order levels that are
    far below the largest one differ by more than 64 eps of themselves.
    Smoothing, the coarsest solve and the V-cycle from the level compare
    with the oracle's in max norm."""
    torch, dev = torch_dev
    m, H = _case(name)
    s = _solver(name)
    rng = np.random.default_rng(3)

    def dev_csr(l, which, shape):
        rp, ci, val = s.level_csr(l, which)
        return sp.csr_matrix((val, ci, rp), shape=shape)

    for l, lv in enumerate(H.levels):
        n = lv.A.shape[0]
        f = rng.standard_normal(n)
        x = rng.standard_normal(n)
        ft, xt = _to(torch, dev, f), _to(torch, dev, x)
        out = torch.zeros(n, dtype=torch.float64, device=dev)
        A = dev_csr(l, "A", lv.A.shape)
        absA = abs(A)
        # product and residual
        s.apply("spmv", l, xt, out=out)
        bound = 64 * EPS * (absA @ np.abs(x)) + 1e-300
        assert np.all(np.abs(out.cpu().numpy() - A @ x) <= bound), f"spmv {l}"
        s.apply("residual", l, ft, xt, out=out)
        assert np.all(np.abs(out.cpu().numpy() - (f - A @ x)) <= bound + 64 * EPS * np.abs(f)), \
            f"residual {l}"
        if l + 1 == len(H.levels):
            s.apply("coarse", l, ft, out=out)
            ref = cycle.coarse_solve(lv, f)
            assert _maxnorm_close(out.cpu().numpy(), ref, 1e-11), "coarse"
            continue
        nc = H.levels[l + 1].A.shape[0]
        R = dev_csr(l, "R", lv.R.shape)
        P = dev_csr(l, "P", lv.P.shape)
        outc = torch.zeros(nc, dtype=torch.float64, device=dev)
        s.apply("restrict", l, ft, out=outc)
        ref = R @ f
        assert np.all(np.abs(outc.cpu().numpy() - ref) <= 64 * EPS * (abs(R) @ np.abs(f)) + 1e-300), \
            f"restrict {l}"
        ec = rng.standard_normal(nc)
        y = xt.clone()
        s.apply("prolong_add", l, _to(torch, dev, ec), out=y)
        ref = x + P @ ec
        assert np.all(np.abs(y.cpu().numpy() - ref) <= 64 * EPS * (np.abs(x) + abs(P) @ np.abs(ec))), \
            f"prolong {l}"
        # smoothing from zero and from an iterate
        s.apply("presmooth", l, ft, out=out)
        ref = cycle.smooth(H, lv, f, None)
        assert _maxnorm_close(out.cpu().numpy(), ref, 1e-11), f"presmooth {l}"
        y = xt.clone()
        s.apply("postsmooth", l, ft, out=y)
        ref = cycle.smooth(H, lv, f, x)
        assert _maxnorm_close(y.cpu().numpy(), ref, 1e-11), f"postsmooth {l}"
        # the whole cycle from this level
        s.apply("vcycle", l, ft, out=out)
        ref = cycle.vcycle(H, f, l)
        assert _maxnorm_close(out.cpu().numpy(), ref, 1e-11), f"vcycle {l}"
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_solve_parity(torch_dev, name):
    torch, dev = torch_dev
    m, H = _case(name)
    b = synth.normal_rhs(m.n_nodes, 12)
    if CASES[name][6] == "pin":
        b = synth.pinned_normal_batch(m.n_nodes, 1, 14)[:, 0].copy()
    s = _solver(name)
    x, info = s.solve(_to(torch, dev, b), tol=1e-10)
    ref = krylov.giamg_pcg(H, b, tol=1e-10)
    assert info.status == 0 and ref.converged
    assert abs(info.iters - ref.iters) <= 1
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    assert info.true_relres < 1e-9
    # fixed iteration count: the stopping boundary plays no part
    k = min(info.iters, ref.iters)
    from paper_2512_15121_amd import Solver, Options
    n_, p, lam, sm, pert, cm, bc, basis, sched = CASES[name]
    s2 = Solver(m.coords, m.l2g, p, lam, Options(smoother=sm, coarse_max=cm, bc=bc, maxit=k,
                                                 basis=basis, schedule=tuple(sched),
                                                 **CASE_OPTS.get(name, {})))
    x2, info2 = s2.solve(_to(torch, dev, b), tol=0.0)
    ref2 = krylov.giamg_pcg(H, b, tol=0.0, maxit=k)
    assert info2.iters == k == ref2.iters
    assert np.linalg.norm(x2.cpu().numpy() - ref2.x) <= 1e-9 * np.linalg.norm(ref2.x)
    assert abs(info2.relres - ref2.history[-1]) <= 1e-6 * ref2.history[-1]
    s.close()
    s2.close()


def test_manufactured_rhs_and_load_vector(torch_dev):
    torch, dev = torch_dev
    name = "manufactured_4cube_p2_jacobi"
    m, H = _case(name)
    s = _solver(name)
    xq = s.quadrature_points()
    xq_o = assembly.quadrature_points(m.coords, m.l2g, 2)
    assert np.max(np.abs(xq - xq_o)) <= 1e-15
    lam = CASES[name][2]
    fq = (lam + 3 * math.pi ** 2) * np.prod(np.sin(math.pi * xq), axis=2)
    b = s.load_vector(fq)
    b_o = assembly.load_vector(m.coords, m.l2g, 2, fq, H.constrained)
    assert np.max(np.abs(b - b_o)) <= 1e-14 * np.max(np.abs(b_o))
    x, info = s.solve(_to(torch, dev, b), tol=1e-10)
    ref = krylov.giamg_pcg(H, b_o, tol=1e-10)
    assert abs(info.iters - ref.iters) <= 1
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    s.close()


@pytest.mark.parametrize("name", ["p4_6cube_cheb_sa", "p4_5cube_cheb1_sa", "p3_6cube_cheb3_sa",
                                  "p6_3cube_cheb4", "p4_4cube_jacobi3", "p8_2cube_keep_boundary"])
def test_mixed_precision_solve(torch_dev, name):
    """FP32 V-cycle inside FP64 flexible CG: the true residual reaches the
    tolerance and the solution is within 1e-8 of the FP64 oracle's."""
    torch, dev = torch_dev
    m, H = _case(name)
    b = synth.normal_rhs(m.n_nodes, 12)
    s = _solver(name, precision="mixed")
    x, info = s.solve(_to(torch, dev, b), tol=1e-10)
    ref = krylov.giamg_pcg(H, b, tol=1e-10)
    assert info.status == 0 and info.true_relres < 1e-9
    err = np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x)
    assert err <= 1e-8, err
    if name != "p4_6cube_cheb_sa":
        s.close()
        return
    # FP32 product of the fine operator: rounding bound (m + 2) 2^-24 (|A||x|)_i
    rng = np.random.default_rng(1)
    lv = H.levels[0]
    xv = rng.standard_normal(lv.A.shape[0])
    out = torch.zeros(lv.A.shape[0], dtype=torch.float32, device=dev)
    s.apply("spmv", 0, _to(torch, dev, xv, torch.float32), out=out, fp32=True)
    mrow = np.diff(lv.A.indptr)
    bound = (mrow + 2) * 2.0 ** -24 * (abs(lv.A) @ np.abs(xv))
    assert np.all(np.abs(out.cpu().numpy().astype(np.float64) - lv.A @ xv) <= bound)
    s.close()


@pytest.mark.parametrize("name", ["p4_6cube_cheb_sa", "p4_5cube_cheb1_sa", "p3_6cube_cheb3_sa",
                                  "p6_3cube_cheb4", "p4_4cube_jacobi3"])
def test_fp32_smoothing_and_vcycle_steps(torch_dev, name):
    """The FP32 operators of a mixed-precision handle, step by step against
    the FP64 oracle in max norm: pre- and post-smoothing (every Chebyshev
    degree's FP32 recurrence) to 1e-5 of the largest entry, a few FP32
    products deep (unit roundoff 6e-8 times the products' row lengths and
    the recurrence's amplification); the V-cycle, whose coarsest solve stays
    FP64, to the same bar."""
    torch, dev = torch_dev
    m, H = _case(name)
    s = _solver(name, precision="mixed")
    rng = np.random.default_rng(5)
    f32 = torch.float32
    for l, lv in enumerate(H.levels[:-1]):
        n = lv.A.shape[0]
        f = rng.standard_normal(n).astype(np.float32).astype(np.float64)
        x = rng.standard_normal(n).astype(np.float32).astype(np.float64)
        ft, xt = _to(torch, dev, f, f32), _to(torch, dev, x, f32)
        out = torch.zeros(n, dtype=f32, device=dev)
        s.apply("presmooth", l, ft, out=out, fp32=True)
        got = out.cpu().numpy().astype(np.float64)
        assert _maxnorm_close(got, cycle.smooth(H, lv, f, None), 1e-5), f"presmooth {l}"
        y = xt.clone()
        s.apply("postsmooth", l, ft, out=y, fp32=True)
        got = y.cpu().numpy().astype(np.float64)
        assert _maxnorm_close(got, cycle.smooth(H, lv, f, x), 1e-5), f"postsmooth {l}"
        s.apply("vcycle", l, ft, out=out, fp32=True)
        got = out.cpu().numpy().astype(np.float64)
        assert _maxnorm_close(got, cycle.vcycle(H, f, l), 1e-5), f"vcycle {l}"
    s.close()


def test_edge_cases(torch_dev):
    torch, dev = torch_dev
    from paper_2512_15121_amd import Solver, Options, giamg
    name = "manufactured_4cube_p2_jacobi"
    m, H = _case(name)
    s = _solver(name)
    n = m.n_nodes
    # zero right-hand side: x = 0 without iterating
    x, info = s.solve(torch.zeros(n, dtype=torch.float64, device=dev),
                      torch.ones(n, dtype=torch.float64, device=dev))
    assert info.iters == 0 and torch.count_nonzero(x).item() == 0
    # initial guess already the solution
    b = synth.normal_rhs(n, 5)
    ref = krylov.giamg_pcg(H, b, tol=1e-13)
    x, info = s.solve(_to(torch, dev, b), _to(torch, dev, ref.x), tol=1e-10)
    assert info.iters == 0
    # non-finite right-hand side: breakdown, reported
    bad = b.copy()
    bad[3] = np.nan
    with pytest.raises(giamg.GiamgError) as e:
        s.solve(_to(torch, dev, bad))
    assert e.value.code == giamg.EBREAKDOWN
    s.close()
    # iteration cap: a warning code, the last iterate returned
    s1 = Solver(m.coords, m.l2g, 2, 1.0, Options(smoother="jacobi", maxit=1))
    x, info = s1.solve(_to(torch, dev, b))
    assert info.status == giamg.ENOTCONV and info.iters == 1
    s1.close()
    # single element of order 2: one free node, one level
    m1 = synth.hex_mesh(1, 2)
    s2 = Solver(m1.coords, m1.l2g, 2, 1.0)
    assert s2.num_levels() == 1
    b1 = synth.normal_rhs(m1.n_nodes, 1)
    x, info = s2.solve(_to(torch, dev, b1))
    H1 = hierarchy.build(m1.coords, m1.l2g, 2, 1.0)
    assert np.allclose(x.cpu().numpy(), np.linalg.solve(H1.levels[0].A.toarray(), b1), rtol=1e-12)
    s2.close()
    # order 1 small enough to be the coarsest level itself
    m3 = synth.hex_mesh(3, 1, perturb=0.1, seed=1)
    s3 = Solver(m3.coords, m3.l2g, 1, 2.0)
    assert s3.num_levels() == 1
    s3.close()
    # bad geometry is rejected with a message
    l2g = m.l2g.copy()
    l2g[0] = l2g[0][::-1]
    with pytest.raises(giamg.GiamgError):
        Solver(m.coords, l2g, 2, 1.0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["p4_6cube_cheb_sa", "manufactured_4cube_p2_jacobi", "p3_pin_neumann"])
def test_graph_replay_equals_eager(torch_dev, name, precision):
    """One CG iteration is captured as a graph at the first solve of a
    handle and replayed.  Replays across several solves, with eager work on
    the same handle and stream syncs between them, give the same iterates,
    bit for bit, as launching every kernel from the host."""
    torch, dev = torch_dev
    m, _ = _case(name)
    n = m.n_nodes
    sg = _solver(name, precision=precision, graph_launch=True)
    se = _solver(name, precision=precision)
    tmp = torch.zeros(n, dtype=torch.float64, device=dev)
    for trial, tol in enumerate([1e-10, 1e-6, 1e-12, 1e-10]):
        if CASES[name][6] == "pin":
            b = synth.pinned_normal_batch(n, 1, 30 + trial)[:, 0].copy()
        else:
            b = synth.normal_rhs(n, 30 + trial)
        bt = _to(torch, dev, b)
        xg, ig = sg.solve(bt, tol=tol)
        xe, ie = se.solve(bt, tol=tol)
        assert ig.status == ie.status == 0 and ig.iters == ie.iters, (trial, ig, ie)
        assert torch.equal(xg, xe), trial
        assert ig.relres == ie.relres
        # eager work on the graph handle and the default stream between replays
        sg.apply("spmv", 0, xg, out=tmp)
        tmp.mul_(0.5)
        torch.cuda.synchronize()
    sg.close()
    se.close()


def test_determinism(torch_dev):
    torch, dev = torch_dev
    name = "p5_7cube_ragged"
    m, H = _case(name)
    b = _to(torch, dev, synth.normal_rhs(m.n_nodes, 3))
    s = _solver(name)
    x1, i1 = s.solve(b)
    x2, i2 = s.solve(b)
    assert i1.iters == i2.iters and torch.equal(x1, x2)
    # Iterations are queued in chunks sized by the previous solve and stop on
    # a device flag: a handle's history changes neither count nor result.
    b2 = _to(torch, dev, synth.normal_rhs(m.n_nodes, 4))
    x3, i3 = s.solve(b2, tol=1e-6)
    x4, i4 = s.solve(b2, tol=1e-12)
    for tol, (xr, ir) in ((1e-6, (x3, i3)), (1e-12, (x4, i4))):
        fresh = _solver(name)
        xf, inf_ = fresh.solve(b2, tol=tol)
        assert ir.iters == inf_.iters and ir.status == inf_.status == 0 and torch.equal(xr, xf)
        fresh.close()
    assert i3.iters < i1.iters < i4.iters
    s.close()


def test_rows_longer_than_a_block(torch_dev):
    """The centre vertex of a 2^3 mesh of order 10 with one pinned node
    couples with 21^3 - 1 = 9260 nodes, more than a row block holds (8192
    nonzeros in FP64 and in FP32): that row gets a block of its own, summed
    by the whole block.  FP64 and FP32 products of the fine operator against
    the oracle's (FP64 to 1e-12 of sum |a_ij x_j|; FP32 within the
    worst-case bound of a 9260-term FP32 sum), and the staged and direct
    forms bit for bit."""
    torch, dev = torch_dev
    from paper_2512_15121_amd import Solver, Options
    m = synth.hex_mesh(2, 10, perturb=0.1, seed=3)
    A, _ = assembly.assemble(m.coords, m.l2g, 10, 1.0, bc="pin")
    A = A.tocsr()
    n, longest = A.shape[0], _max_row(A)
    assert longest == 21 ** 3 - 1
    x = np.random.default_rng(21).standard_normal(n)
    ref, bound = A @ x, abs(A) @ np.abs(x)
    xt = _to(torch, dev, x)
    outs = {}
    for name, kw in (("mixed", {"precision": "mixed"}), ("direct", {"direct_gathers": 1})):
        s = Solver(m.coords, m.l2g, 10, 1.0, Options(bc="pin", **kw))
        y = torch.zeros(n, dtype=torch.float64, device=dev)
        s.apply("spmv", 0, xt, out=y)
        outs[name] = y
        yh = y.cpu().numpy()
        assert np.all(np.abs(yh - ref) <= 1e-12 * bound), name
        if name == "mixed":
            x32 = x.astype(np.float32)
            A32 = sp.csr_matrix((A.data.astype(np.float32).astype(np.float64), A.indices, A.indptr), A.shape)
            ref32 = A32 @ x32.astype(np.float64)
            bound32 = abs(A32) @ np.abs(x32.astype(np.float64))
            y32 = torch.zeros(n, dtype=torch.float32, device=dev)
            s.apply("spmv", 0, _to(torch, dev, x32), out=y32, fp32=True)
            err = np.abs(y32.cpu().numpy().astype(np.float64) - ref32)
            assert np.all(err <= (longest + 2) * 2.0 ** -24 * bound32)
        s.close()
    assert torch.equal(outs["mixed"], outs["direct"])


def test_hierarchy_info_through_the_c_abi(torch_dev):
    """giamg_hierarchy_info called through ctypes on a live handle: level
    count, rows and nonzeros of every level equal the oracle hierarchy's;
    cap limits what is written; bad arguments are rejected."""
    import ctypes
    from paper_2512_15121_amd import giamg
    name = "p4_6cube_theta"
    m, H = _case(name)
    s = _solver(name)
    lib = giamg.library()
    nl = ctypes.c_int32()
    assert lib.giamg_hierarchy_info(s._h, ctypes.byref(nl), None, None, 0) == giamg.OK
    assert nl.value == len(H.levels)
    rows = np.full(nl.value + 2, -1, dtype=np.int64)
    nnz = np.full(nl.value + 2, -1, dtype=np.int64)
    assert lib.giamg_hierarchy_info(s._h, ctypes.byref(nl), giamg._ptr(rows), giamg._ptr(nnz),
                                    nl.value + 2) == giamg.OK
    assert list(rows[:nl.value]) == [lv.A.shape[0] for lv in H.levels]
    assert list(nnz[:nl.value]) == [lv.A.nnz for lv in H.levels]
    assert (rows[nl.value:] == -1).all() and (nnz[nl.value:] == -1).all()
    rows2 = np.full(2, -1, dtype=np.int64)
    nnz2 = np.full(2, -1, dtype=np.int64)
    assert lib.giamg_hierarchy_info(s._h, ctypes.byref(nl), giamg._ptr(rows2), giamg._ptr(nnz2),
                                    1) == giamg.OK
    assert rows2[0] == rows[0] and rows2[1] == -1 and nl.value == len(H.levels)
    assert lib.giamg_hierarchy_info(s._h, ctypes.byref(nl), None, None, 3) == giamg.EINVAL
    assert lib.giamg_hierarchy_info(s._h, ctypes.byref(nl), None, None, -1) == giamg.EINVAL
    r, z = s.hierarchy_info()
    assert list(r) == list(rows[:nl.value]) and list(z) == list(nnz[:nl.value])
    # the strength threshold changed the aggregation: more aggregates than at theta = 0
    H0 = hierarchy.build(m.coords, m.l2g, 4, 10.0, hierarchy.Options(coarse_max=100))
    assert H.levels[-1].A.shape[0] > H0.levels[-1].A.shape[0]
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_profile_counts_and_unchanged_results(torch_dev, precision):
    """Phase profiling (the paper's breakdown categories): a solve of k CG
    iterations with Chebyshev degree 2 runs k V-cycles (the start-up one and
    k - 1 in the loop: the converged iteration skips its second half), two
    fine-level Chebyshev steps per V-cycle, k CG products; work queued past
    convergence is not counted.  Profiling changes no result bit, and the
    phases fit inside the solve's own time."""
    torch, dev = torch_dev
    name = "p4_6cube_cheb_sa"
    m, H = _case(name)
    b = _to(torch, dev, synth.normal_rhs(m.n_nodes, 12))
    s = _solver(name, precision=precision)
    x0, i0 = s.solve(b, tol=1e-10)
    s.profile(True)
    total_ms = 0.0
    for _ in range(2):
        x1, i1 = s.solve(b, tol=1e-10)
        total_ms += i1.solve_ms
        assert torch.equal(x1, x0) and i1.iters == i0.iters
    p = s.profile_read(reset=True)
    s.profile(False)
    k = i0.iters
    assert p["solves"] == 2 and p["iterations"] == 2 * k
    assert p["vcycle"][1] == 2 * k and p["pcg"][1] == 2 * k and p["cg_matvec"][1] == 2 * k
    assert p["fine_step"][1] == 2 * 2 * k
    assert p["first_smooth"][1] == 2 * 2 * k
    nl = s.num_levels()
    assert p["coarse"][1] == 2 * k
    assert p["smooth"][1] == 2 * 2 * k * (nl - 1)
    for ph in ("first_smooth", "smooth", "residual", "transfer", "coarse", "vcycle", "cg_matvec",
               "cg_dot", "cg_update", "pcg", "fine_step"):
        assert p[ph][0] > 0, ph
    assert p["pcg"][0] <= total_ms and p["vcycle"][0] <= total_ms
    assert p["first_smooth"][0] <= p["smooth"][0] + 1e-6
    assert p["fine_step"][0] <= p["first_smooth"][0] + 1e-6
    # reading again after the reset: empty
    q = s.profile_read(reset=False)
    assert q["solves"] == 0 and q["vcycle"] == (0.0, 0)
    s.close()


def test_kernel_timing_and_read_bandwidth(torch_dev):
    """The measurement entry points: every kernel kind of giamg_time_kernel
    runs on the fine level and reports a positive duration and its bytes
    (the CG product in FP64 only), the solve is unchanged by them, and the
    read-stream reference reports a positive rate."""
    torch, dev = torch_dev
    from paper_2512_15121_amd import giamg
    name = "p4_6cube_cheb_sa"
    m, H = _case(name)
    b = _to(torch, dev, synth.normal_rhs(m.n_nodes, 12))
    s = _solver(name, precision="mixed")
    x0, i0 = s.solve(b, tol=1e-10)
    n0, nnz0 = s.level(0)["rows"], s.level(0)["nnz_A"]
    for kind in ("cheb_step", "spmv", "restrict", "prolong", "cg_product"):
        ms, by = s.time_kernel(kind, level=0, reps=3)
        assert ms > 0 and by > 0, kind
        if kind in ("cheb_step", "spmv", "cg_product"):
            assert by >= 8 * nnz0 + 8 * n0, kind
    ms, by = s.time_kernel("cheb_step", level=0, reps=3, fp32=True)
    assert ms > 0 and 4 * nnz0 <= by
    with pytest.raises(giamg.GiamgError):
        s.time_kernel("cg_product", level=0, reps=3, fp32=True)
    x1, i1 = s.solve(b, tol=1e-10)
    assert torch.equal(x1, x0) and i1.iters == i0.iters
    s.close()
    assert giamg.read_bandwidth(1 << 24, 3) > 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_initial_guess_skips_the_product_with_the_same_bits(torch_dev, precision):
    """A zero initial guess is detected on the device and the first residual
    is b itself, without the product A x: the solve equals, bit for bit, the
    one started from -0 everywhere (a nonzero bit pattern, so the product is
    formed), and a nonzero guess is still honoured."""
    torch, dev = torch_dev
    name = "p4_6cube_cheb_sa"
    m, H = _case(name)
    b = _to(torch, dev, synth.normal_rhs(m.n_nodes, 31))
    s = _solver(name, precision=precision)
    x0 = torch.zeros_like(b)
    xa, ia = s.solve(b, x0.clone(), tol=1e-10)
    xb, ib = s.solve(b, torch.full_like(b, -0.0), tol=1e-10)
    assert ia.iters == ib.iters and torch.equal(xa, xb)
    assert ia.true_relres < 1e-9
    # a converged guess: no iterations, unchanged
    xc, ic = s.solve(b, xa.clone(), tol=1e-6)
    assert ic.iters == 0 and torch.equal(xc, xa)
    s.close()


def test_jacobi_pcg_baseline_parity(torch_dev):
    """The diagonally preconditioned CG baseline of the paper's comparison
    (Section 3.2): one level, against the oracle's Jacobi-PCG.  A run of a
    fixed number of iterations matches to 1e-9 (iterate) and 1e-6
    (recursive residual); to the tolerance the iteration counts agree within
    one percent (hundreds of iterations let rounding move the stopping point
    by one or two).  The V-cycle-only entry points refuse such a handle."""
    torch, dev = torch_dev
    from paper_2512_15121_amd import giamg
    name = "p4_6cube_cheb_sa"
    m, H = _case(name)
    A = H.levels[0].A
    b = synth.normal_rhs(m.n_nodes, 12)
    bt = _to(torch, dev, b)
    s = _solver(name, preconditioner="jacobi")
    assert s.num_levels() == 1
    x, info = s.solve(bt, tol=1e-10)
    ref = krylov.jacobi_pcg(A, b, tol=1e-10)
    assert info.status == 0 and ref.converged and ref.iters > 50
    assert abs(info.iters - ref.iters) <= max(1, ref.iters // 100), (info.iters, ref.iters)
    assert info.true_relres < 2e-10
    k = 40
    s2 = _solver(name, preconditioner="jacobi", maxit=k)
    x2, i2 = s2.solve(bt, tol=0.0)
    ref2 = krylov.jacobi_pcg(A, b, tol=0.0, maxit=k)
    assert i2.iters == k == ref2.iters
    assert np.linalg.norm(x2.cpu().numpy() - ref2.x) <= 1e-9 * np.linalg.norm(ref2.x)
    assert abs(i2.relres - ref2.history[-1]) <= 1e-6 * ref2.history[-1]
    with pytest.raises(giamg.GiamgError) as e:
        s.solve_batch(torch.zeros(m.n_nodes, 2, dtype=torch.float64, device=dev))
    assert e.value.code == giamg.ENOTSUP
    s.close()
    s2.close()
    with pytest.raises(giamg.GiamgError) as e:
        _solver(name, preconditioner="jacobi", precision="mixed")
    assert e.value.code == giamg.EINVAL
