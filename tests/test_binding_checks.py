"""The binding checks every tensor it hands to the C ABI as a bare pointer
(dtype, shape, contiguity, device) and raises ValueError before any library
call: a float32 or short tensor would otherwise let a kernel read or write
past the buffer.  No GPU: the solver objects are built without a handle and
with a library stand-in that fails the test if it is reached."""
import numpy as np
import pytest
import torch

from paper_2512_15121_amd import giamg


class _NoLibrary:
    def __getattr__(self, name):
        def call(*args):
            raise AssertionError(f"library entry point {name} reached")
        return call


def _solver(n_nodes=10, rows=(10, 3)):
    s = giamg.Solver.__new__(giamg.Solver)
    s.lib = _NoLibrary()
    s._h = None
    s.n_nodes = n_nodes
    s.num_levels = lambda: len(rows)
    s.level = lambda l: {"rows": rows[l]}
    return s


def test_solve_rejects_dtype_shape_and_host_tensors():
    s = _solver()
    with pytest.raises(ValueError, match="dtype"):
        s.solve(torch.zeros(10, dtype=torch.float32), torch.zeros(10, dtype=torch.float32))
    with pytest.raises(ValueError, match="shape"):
        s.solve(torch.zeros(9, dtype=torch.float64), torch.zeros(9, dtype=torch.float64))
    with pytest.raises(ValueError, match="shape"):
        s.solve(torch.zeros(10, dtype=torch.float64), torch.zeros(11, dtype=torch.float64))
    with pytest.raises(ValueError, match="contiguous"):
        s.solve(torch.zeros(20, dtype=torch.float64)[::2], torch.zeros(10, dtype=torch.float64))
    with pytest.raises(ValueError, match="device"):
        s.solve(torch.zeros(10, dtype=torch.float64), torch.zeros(10, dtype=torch.float64))
    with pytest.raises(ValueError, match="torch tensor"):
        s.solve(np.zeros(10), torch.zeros(10, dtype=torch.float64))


def test_solve_batch_rejects_mismatched_blocks():
    s = _solver()
    with pytest.raises(ValueError, match="2-D"):
        s.solve_batch(torch.zeros(10, dtype=torch.float64))
    with pytest.raises(ValueError, match="shape"):
        s.solve_batch(torch.zeros(10, 4, dtype=torch.float64), torch.zeros(10, 3, dtype=torch.float64))
    with pytest.raises(ValueError, match="shape"):
        s.solve_batch(torch.zeros(12, 4, dtype=torch.float64))
    with pytest.raises(ValueError, match="dtype"):
        s.solve_batch(torch.zeros(10, 4, dtype=torch.float32))
    with pytest.raises(ValueError, match="contiguous"):
        s.solve_batch(torch.zeros(4, 10, dtype=torch.float64).t())


def test_apply_sizes_vectors_by_level():
    s = _solver()
    f64 = torch.float64
    with pytest.raises(ValueError, match="^out:"):    # restrict writes the coarse level
        s.apply("restrict", 0, torch.zeros(10, dtype=f64), out=torch.zeros(10, dtype=f64))
    with pytest.raises(ValueError, match="^a:"):      # prolong reads the coarse level
        s.apply("prolong_add", 0, torch.zeros(10, dtype=f64), out=torch.zeros(10, dtype=f64))
    with pytest.raises(ValueError, match="dtype"):
        s.apply("spmv", 0, torch.zeros(10, dtype=f64), out=torch.zeros(10, dtype=f64), fp32=True)
    with pytest.raises(ValueError, match="needs b"):
        s.apply("residual", 0, torch.zeros(10, dtype=f64), out=torch.zeros(10, dtype=f64))
    with pytest.raises(ValueError, match="coarser level"):
        s.apply("restrict", 1, torch.zeros(3, dtype=f64), out=torch.zeros(3, dtype=f64))
    with pytest.raises(ValueError, match="out of range"):
        s.apply("spmv", 2, torch.zeros(3, dtype=f64), out=torch.zeros(3, dtype=f64))
    # right sizes and dtype reach the device check (host tensors here)
    with pytest.raises(ValueError, match="device"):
        s.apply("restrict", 0, torch.zeros(10, dtype=f64), out=torch.zeros(3, dtype=f64))


def test_session_admit_and_retire_check_their_tensors():
    sess = giamg.Session.__new__(giamg.Session)
    sess.lib = _NoLibrary()
    sess.solver = _solver()
    sess.slots = 4
    sess._s = None
    sess._keep = {}
    with pytest.raises(ValueError, match="dtype"):
        sess.admit([0], [torch.zeros(10, dtype=torch.float32)])
    with pytest.raises(ValueError, match="shape"):
        sess.admit([0], [torch.zeros(7, dtype=torch.float64)])
    with pytest.raises(ValueError, match="slot"):
        sess.admit([4], [torch.zeros(10, dtype=torch.float64)])
    with pytest.raises(ValueError, match="same length"):
        sess.admit([0, 1], [torch.zeros(10, dtype=torch.float64)])
    with pytest.raises(ValueError, match="device"):
        sess.admit([0], [torch.zeros(10, dtype=torch.float64)])
    with pytest.raises(ValueError, match="shape"):
        sess.retire(0, torch.zeros(9, dtype=torch.float64))


def test_server_submit_checks_size():
    srv = giamg.Server.__new__(giamg.Server)
    srv.lib = _NoLibrary()
    srv._s = None
    srv._sizes = [10]
    srv._out = {}
    with pytest.raises(ValueError, match="entries"):
        srv.submit(0, np.zeros(9))
    with pytest.raises(ValueError, match="unknown problem"):
        srv.submit(1, np.zeros(10))
