"""giamg_solve_noalloc, the solve whose CG work vectors live in the
library's fixed per-GPU scratch array, called through the C ABI (ctypes):

* two calls in a row, the second on a smaller problem (a smaller handle), in
  FP64 and mixed precision: iterations, status, residuals and the solution
  equal giamg_solve's bit for bit (same kernels, same reduction order);
* no device allocation through the library's allocator during the calls
  (a counting allocator is registered before the handles are built);
* a problem larger than the scratch is rejected with GIAMG_EINVAL and a
  message, and x is left untouched.
"""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _noalloc(lib, h, b, x, tol):
    from paper_2512_15121_amd import giamg
    info = giamg._Info()
    rc = lib.giamg_solve_noalloc(h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                 tol, ctypes.byref(info))
    return rc, info


def test_noalloc_solve_equals_solve_and_allocates_nothing():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2512_15121_amd import giamg, Solver, Options
    lib = giamg.library()
    dev = torch.device("cuda:0")
    counts = {"alloc": 0}

    def alloc(nbytes, stream):
        counts["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(nbytes, 0, stream)

    giamg.set_allocator(alloc, lambda p: torch.cuda.caching_allocator_delete(p))
    try:
        cases = [(10, 4, 10.0, 3), (5, 3, 1.0, 4)]      # the second call is smaller
        for precision in ("fp64", "mixed"):
            solvers = []
            for n, p, lam, seed in cases:
                m = synth.hex_mesh(n, p, perturb=0.1, seed=seed)
                s = Solver(m.coords, m.l2g, p, lam, Options(precision=precision, coarse_max=300))
                b = torch.from_numpy(synth.normal_rhs(m.n_nodes, 60 + seed)).to(dev)
                solvers.append((s, b))
            assert solvers[1][0].n_nodes < solvers[0][0].n_nodes
            torch.cuda.synchronize()
            for s, b in solvers:
                x_ref, i_ref = s.solve(b, tol=1e-10)
                x = torch.zeros_like(b)
                torch.cuda.synchronize()
                before = counts["alloc"]
                rc, info = _noalloc(lib, s._h, b, x, 1e-10)
                assert counts["alloc"] == before, "the no-allocation solve allocated"
                assert rc == giamg.OK, lib.giamg_last_error()
                assert info.iters == i_ref.iters and info.status == i_ref.status == 0
                assert info.relres == i_ref.relres and info.true_relres == i_ref.true_relres
                assert info.true_relres < 1e-9
                assert torch.equal(x, x_ref), precision
            for s, _ in solvers:
                s.close()
        # a problem larger than the scratch: rejected, nothing written
        m = synth.hex_mesh(22, 4, perturb=0.1, seed=5)          # 89^3 = 704,969 nodes
        big = Solver(m.coords, m.l2g, 4, 1.0, Options())
        b = torch.from_numpy(synth.normal_rhs(m.n_nodes, 9)).to(dev)
        x = torch.full_like(b, 3.0)
        rc, _ = _noalloc(lib, big._h, b, x, 1e-10)
        assert rc == giamg.EINVAL and b"scratch" in lib.giamg_last_error()
        assert torch.all(x == 3.0)
        big.close()
    finally:
        giamg.set_allocator()
