"""Device memory through a caller's allocator (giamg_set_allocator): every
block the library takes comes from the registered allocator and goes back
to it, and results do not depend on where the memory came from."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_torch_allocator_routes_all_device_memory():
    import torch
    from paper_2512_15121_amd import Solver, Options, giamg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m = synth.hex_mesh(5, 3, perturb=0.1, seed=4)
    b = torch.from_numpy(synth.normal_rhs(m.n_nodes, 3)).to("cuda:0")
    B = torch.from_numpy(synth.normal_rhs(m.n_nodes * 4, 5).reshape(m.n_nodes, 4)).to("cuda:0")
    live, total = {}, [0, 0]

    def alloc(n, stream):
        p = torch.cuda.caching_allocator_alloc(n, 0, stream)
        live[p] = n
        total[0] += 1
        total[1] += n
        return p

    def release(p):
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    giamg.set_allocator(alloc, release)
    try:
        s = Solver(m.coords, m.l2g, 3, 2.0, Options(precision="mixed"))
        after_setup = total[0]
        x1, i1 = s.solve(b, tol=1e-10)
        X1, _ = s.solve_batch(B, tol=1e-10)
        torch.cuda.synchronize()
        assert after_setup > 10 and total[0] >= after_setup and live
        assert all(p % 256 == 0 for p in live)
        s.close()
        assert live == {}, f"{len(live)} blocks not returned"
    finally:
        giamg.set_allocator()
    s2 = Solver(m.coords, m.l2g, 3, 2.0, Options(precision="mixed"))
    x2, i2 = s2.solve(b, tol=1e-10)
    X2, _ = s2.solve_batch(B, tol=1e-10)
    assert i1.iters == i2.iters and torch.equal(x1, x2) and torch.equal(X1, X2)
    s2.close()
    n_before = total[0]
    s3 = Solver(m.coords, m.l2g, 3, 2.0, Options())   # hipMalloc again
    s3.close()
    assert total[0] == n_before


def test_failing_allocator_is_an_allocation_error():
    import torch
    from paper_2512_15121_amd import Solver, Options, giamg
    m = synth.hex_mesh(3, 2, seed=1)
    giamg.set_allocator(lambda n, s: 0, lambda p: None)
    try:
        with pytest.raises(giamg.GiamgError) as e:
            Solver(m.coords, m.l2g, 2, 1.0, Options())
        assert e.value.code == giamg.ENOMEM
    finally:
        giamg.set_allocator()
    s = Solver(m.coords, m.l2g, 2, 1.0, Options())
    s.close()
