"""Thin ctypes binding of ``libgiamg.so`` (the C ABI in include/giamg.h).

Argument marshalling only: every step of the setup and solve runs inside the
library.  PyTorch provides device memory (CUDA/HIP tensors) and the stream;
results stay on the device.  The binding fails loudly when the library has
not been built -- there is no fallback implementation.
"""
import ctypes
import os
from dataclasses import dataclass, asdict

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgiamg.so")

OK, ENOTCONV, EINVAL, ENOMEM, EHIP, EBREAKDOWN, ENOTSUP = 0, 1, -1, -2, -3, -4, -5
SMOOTHER = {"chebyshev": 0, "jacobi": 1}
BC = {"dirichlet": 0, "pin": 1}
PRECISION = {"fp64": 0, "mixed": 1}
LEVEL_KIND = {0: "p", 1: "h"}
MAT = {"A": 0, "P": 1, "R": 2, "AP": 3}
BASIS = {"nodal": 0, "modal": 1}
PRECONDITIONER = {"vcycle": 0, "jacobi": 1}
ASSEMBLY = {"auto": 0, "device": 1, "host": 2}
BATCH_KERNEL = {"auto": 0, "lanes": 1, "wave": 2, "group": 3}
OP = {"spmv": 0, "residual": 1, "restrict": 2, "prolong_add": 3, "presmooth": 4,
      "postsmooth": 5, "coarse": 6, "vcycle": 7}
OP_FP32 = 256


class GiamgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"giamg error {code}: {msg}")
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [("smoother", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("omega", ctypes.c_double), ("coarse_max", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("pin_node", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("maxit", ctypes.c_int32), ("agg_seed", ctypes.c_uint64),
                ("power_iters", ctypes.c_int32), ("cheb_lo", ctypes.c_double),
                ("cheb_hi", ctypes.c_double), ("direct_gathers", ctypes.c_int32),
                ("graph_launch", ctypes.c_int32), ("basis", ctypes.c_int32),
                ("schedule", ctypes.c_int32 * 8), ("batch_kernel", ctypes.c_int32),
                ("row_groups", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("lean_max_nnz", ctypes.c_int64), ("keep_boundary", ctypes.c_int32),
                ("pad2", ctypes.c_int32), ("theta", ctypes.c_double),
                ("preconditioner", ctypes.c_int32), ("assembly", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("relres", ctypes.c_double), ("true_relres", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("slots", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("tol", ctypes.c_double),
                ("hold_ms", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("setups", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("cache_hits", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("resident_bytes", ctypes.c_int64), ("groups_resident", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


PHASES = ["first_smooth", "smooth", "residual", "transfer", "coarse", "vcycle", "cg_matvec",
          "cg_dot", "cg_update", "pcg", "fine_step"]


class _Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(PHASES)), ("count", ctypes.c_int64 * len(PHASES)),
                ("solves", ctypes.c_int64), ("iterations", ctypes.c_int64)]


class _LevelDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("order", ctypes.c_int32),
                ("coarsest", ctypes.c_int32), ("device_assembly", ctypes.c_int32),
                ("rows", ctypes.c_int64), ("nnz_A", ctypes.c_int64),
                ("nnz_P", ctypes.c_int64), ("nnz_R", ctypes.c_int64),
                ("lam_hat", ctypes.c_double), ("nnz_AP", ctypes.c_int64),
                ("staged_nnz_A", ctypes.c_int64), ("runs_A", ctypes.c_int64),
                ("groups_A", ctypes.c_int64), ("group_entries_A", ctypes.c_int64),
                ("lean_A", ctypes.c_int64)]


@dataclass
class Options:
    smoother: str = "chebyshev"
    degree: int = 2
    omega: float = 2.0 / 3.0
    coarse_max: int = 2000
    max_levels: int = 10
    bc: str = "dirichlet"
    pin_node: int = 0
    precision: str = "fp64"
    maxit: int = 500
    agg_seed: int = 0
    power_iters: int = 20
    cheb_lo: float = 0.1
    cheb_hi: float = 1.1
    direct_gathers: bool = False
    graph_launch: bool = False
    basis: str = "nodal"            # or "modal"
    schedule: tuple = ()            # coarse p-orders after p, e.g. (4, 3, 2, 1); () = default
    batch_kernel: str = "auto"      # block-product shape of solve_batch: auto, lanes, wave, group
    row_groups: bool = False        # grouped product form where rows share column lists
    lean_max_nnz: int = 2000000     # row-direct kernel for operators up to this many nonzeros
    keep_boundary: bool = False     # coarse p-levels keep the constrained nodes
    theta: float = 0.0              # strength threshold of the aggregation graph
    preconditioner: str = "vcycle"  # or "jacobi": the diagonally preconditioned CG baseline
    assembly: str = "auto"          # fine operator built on the device where it fits, or "device", "host"

    def _c(self) -> _Opts:
        d = asdict(self)
        d["basis"] = BASIS[d["basis"]]
        d["batch_kernel"] = BATCH_KERNEL[d["batch_kernel"]]
        sched = [int(q) for q in d["schedule"]]
        if len(sched) > 8:
            raise ValueError("at most 8 coarse orders")
        d["schedule"] = (ctypes.c_int32 * 8)(*(sched + [0] * (8 - len(sched))))
        d["direct_gathers"] = int(d["direct_gathers"])
        d["graph_launch"] = int(d["graph_launch"])
        d["row_groups"] = int(d["row_groups"])
        d["pad"] = 0
        d["pad2"] = 0
        d["keep_boundary"] = int(d["keep_boundary"])
        d["preconditioner"] = PRECONDITIONER[d["preconditioner"]]
        d["assembly"] = ASSEMBLY[d["assembly"]]
        d["smoother"] = SMOOTHER[d["smoother"]]
        d["bc"] = BC[d["bc"]]
        d["precision"] = PRECISION[d["precision"]]
        return _Opts(**d)


@dataclass
class SolveInfo:
    iters: int
    status: int
    relres: float
    true_relres: float
    solve_ms: float
    bytes: float


_lib = None

P = ctypes.c_void_p
I32, I64, F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_SIGNATURES = {
    "giamg_set_allocator": (I32, [ALLOC_FN, RELEASE_FN, P]),
    "giamg_default_opts": (None, [ctypes.POINTER(_Opts)]),
    "giamg_setup": (I32, [P, I64, P, I64, I32, F64, ctypes.POINTER(_Opts), P, ctypes.POINTER(P)]),
    "giamg_free": (None, [P]),
    "giamg_solve": (I32, [P, P, P, F64, ctypes.POINTER(_Info)]),
    "giamg_solve_noalloc": (I32, [P, P, P, F64, ctypes.POINTER(_Info)]),
    "giamg_solve_batch": (I32, [P, P, P, I32, F64, ctypes.POINTER(_Info)]),
    "giamg_hierarchy_info": (I32, [P, P, P, P, I32]),
    "giamg_num_levels": (I32, [P]),
    "giamg_level_describe": (I32, [P, I32, ctypes.POINTER(_LevelDesc)]),
    "giamg_level_csr": (I32, [P, I32, I32, P, P, P]),
    "giamg_level_l2g": (I32, [P, I32, P]),
    "giamg_level_aggregates": (I32, [P, I32, P]),
    "giamg_constrained": (I32, [P, P]),
    "giamg_apply": (I32, [P, I32, I32, P, P, P]),
    "giamg_quadrature_points": (I32, [P, P]),
    "giamg_load_vector": (I32, [P, P, P]),
    "giamg_setup_times": (I32, [P, P]),
    "giamg_last_error": (ctypes.c_char_p, []),
    "giamg_profile_enable": (I32, [P, I32]),
    "giamg_profile_read": (I32, [P, ctypes.POINTER(_Profile), I32]),
    "giamg_read_bandwidth": (I32, [I64, I32, P]),
    "giamg_hcsr_size": (I32, [P, P, P, P]),
    "giamg_hcsr_copy": (I32, [P, P, P, P]),
    "giamg_hcsr_free": (None, [P]),
    "giamg_host_boundary": (I32, [P, I64, I32, I64, I32, P]),
    "giamg_host_assemble": (I32, [P, I64, P, I64, I32, F64, I32, I64, I32, ctypes.POINTER(P)]),
    "giamg_host_p_transfer": (I32, [P, I64, I32, I32, I64, P, I32, P, P, ctypes.POINTER(P)]),
    "giamg_host_aggregate": (I32, [P, P, P, I64, ctypes.c_uint64, F64, P, P, ctypes.POINTER(P)]),
    "giamg_host_coarse_inverse": (I32, [P, I64, P]),
    "giamg_time_kernel": (I32, [P, I32, I32, I32, P, P]),
    "giamg_session_create": (I32, [P, I32, F64, ctypes.POINTER(P)]),
    "giamg_session_admit": (I32, [P, I32, P, P]),
    "giamg_session_step": (I32, [P, I32]),
    "giamg_session_poll": (I32, [P, P, P]),
    "giamg_session_retire": (I32, [P, I32, P]),
    "giamg_session_free": (None, [P]),
    "giamg_server_create": (I32, [P, ctypes.POINTER(P)]),
    "giamg_server_add_problem": (I32, [P, P, I64, P, I64, I32, F64, ctypes.POINTER(_Opts), P]),
    "giamg_server_submit": (I32, [P, I32, P, P, P]),
    "giamg_server_wait": (I32, [P, I64, P, P]),
    "giamg_server_stats": (I32, [P, P]),
    "giamg_server_free": (None, [P]),
}
KERNEL = {"cheb_step": 0, "spmv": 1, "restrict": 2, "prolong": 3, "cg_product": 4}


def library() -> ctypes.CDLL:
    """Load libgiamg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


_allocator_refs = None   # the registered callbacks, kept alive while registered


def set_allocator(alloc=None, release=None):
    """Route the library's device memory through alloc(bytes, stream) -> int
    and release(ptr) (Python callables; stream is the hipStream_t as an int,
    0 for the null stream).  With no arguments hipMalloc / hipFree return.
    Blocks allocated before a change go back through the allocator they
    came from."""
    global _allocator_refs
    lib = library()
    if alloc is None and release is None:
        _check(lib.giamg_set_allocator(ALLOC_FN(), RELEASE_FN(), None))
        return

    def _alloc(nbytes, stream, ctx):
        try:
            return int(alloc(int(nbytes), int(stream or 0))) or None
        except Exception:   # reported to the library as an allocation failure
            return None

    def _release(ptr, ctx):
        release(int(ptr))

    refs = (ALLOC_FN(_alloc), RELEASE_FN(_release))
    _check(lib.giamg_set_allocator(refs[0], refs[1], None))
    # keep the previous callbacks alive too: blocks they allocated are
    # released through them
    _allocator_refs = (refs, _allocator_refs)


def use_torch_allocator(device=0):
    """Take the library's device memory from torch's caching allocator on
    `device` (the stream of the allocating handle is passed along)."""
    import torch
    set_allocator(lambda n, s: torch.cuda.caching_allocator_alloc(n, device, s),
                  lambda p: torch.cuda.caching_allocator_delete(p))


def _check(rc):
    if rc < 0 or rc == ENOTCONV:
        msg = library().giamg_last_error().decode()
        if rc < 0:
            raise GiamgError(rc, msg)
    return rc


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _devs(*specs):
    """Device pointers of the tensors in ``specs`` -- (tensor, torch dtype,
    shape, name) each -- after checking what the library will read or write
    through them: the C ABI takes bare pointers, so a wrong dtype or size
    would make a kernel run past the buffer.  Every tensor's dtype, shape
    and layout are checked before any device check, so the error names the
    mismatch."""
    import torch
    for t, dtype, shape, name in specs:
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
        if t.dtype != dtype:
            raise ValueError(f"{name}: expected dtype {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous tensor")
    for t, _, _, name in specs:
        if not t.is_cuda:
            raise ValueError(f"{name}: expected a device tensor, got one on {t.device}")
    return [ctypes.c_void_p(t.data_ptr()) for t, _, _, _ in specs]


class Solver:
    """GIAMG-PCG solver for A = K + lambda M on a hexahedral mesh.

    coords: float64 [n_nodes, 3]; l2g: int32 [n_elem, (p+1)^3] in the tensor
    ordering (p+1)^2 i + (p+1) j + k.  Device work runs on ``stream`` (a
    torch.cuda.Stream, default: the current stream).
    """

    def __init__(self, coords, l2g, p, lam, opts: Options = None, stream=None):
        import torch
        self.lib = library()
        self.opts = opts or Options()
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        l2g = np.ascontiguousarray(l2g, dtype=np.int32)
        self.n_nodes = coords.shape[0]
        self.n_elem = l2g.shape[0]
        self.p = int(p)
        self.stream = stream or torch.cuda.current_stream()
        self._h = ctypes.c_void_p()
        co = self.opts._c()
        _check(self.lib.giamg_setup(_ptr(coords), self.n_nodes, _ptr(l2g), self.n_elem,
                                    self.p, float(lam), ctypes.byref(co),
                                    ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(self._h)))

    def close(self):
        if self._h:
            self.lib.giamg_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- solves --------------------------------------------------------------
    def solve(self, b, x=None, tol=1e-10):
        """b, x: float64 device tensors of n_nodes entries (x: initial guess,
        overwritten with the solution; zeros when omitted)."""
        import torch
        if x is None:
            x = torch.zeros_like(b)
        n = (self.n_nodes,)
        bp, xp = _devs((b, torch.float64, n, "b"), (x, torch.float64, n, "x"))
        info = _Info()
        rc = self.lib.giamg_solve(self._h, bp, xp, float(tol), ctypes.byref(info))
        _check(rc)
        return x, SolveInfo(info.iters, info.status, info.relres, info.true_relres, info.solve_ms, info.bytes)

    def solve_noalloc(self, b, x, tol=1e-10):
        """giamg_solve_noalloc: the solve with its work vectors in the
        library's fixed per-GPU scratch (no allocation; x is required)."""
        import torch
        n = (self.n_nodes,)
        bp, xp = _devs((b, torch.float64, n, "b"), (x, torch.float64, n, "x"))
        info = _Info()
        rc = self.lib.giamg_solve_noalloc(self._h, bp, xp, float(tol), ctypes.byref(info))
        _check(rc)
        return x, SolveInfo(info.iters, info.status, info.relres, info.true_relres, info.solve_ms,
                            info.bytes)

    def solve_batch(self, B, X=None, tol=1e-10):
        """B, X: float64 device tensors [n_nodes, k], right-hand side j in
        column j (X: initial guesses, overwritten)."""
        import torch
        if X is None:
            X = torch.zeros_like(B)
        if not isinstance(B, torch.Tensor) or B.dim() != 2 or B.shape[1] < 1:
            raise ValueError("B: expected a 2-D tensor [n_nodes, k] with k >= 1")
        k = int(B.shape[1])
        shape = (self.n_nodes, k)
        Bp, Xp = _devs((B, torch.float64, shape, "B"), (X, torch.float64, shape, "X"))
        infos = (_Info * k)()
        rc = self.lib.giamg_solve_batch(self._h, Bp, Xp, k, float(tol), infos)
        _check(rc)
        return X, [SolveInfo(i.iters, i.status, i.relres, i.true_relres, i.solve_ms, i.bytes) for i in infos]

    # -- introspection -------------------------------------------------------
    def num_levels(self) -> int:
        return _check(self.lib.giamg_num_levels(self._h))

    def hierarchy_info(self):
        """(rows, nnz) of A on every level, fine level first."""
        nl = ctypes.c_int32()
        _check(self.lib.giamg_hierarchy_info(self._h, ctypes.byref(nl), None, None, 0))
        rows = np.zeros(nl.value, dtype=np.int64)
        nnz = np.zeros(nl.value, dtype=np.int64)
        _check(self.lib.giamg_hierarchy_info(self._h, ctypes.byref(nl), _ptr(rows), _ptr(nnz),
                                             nl.value))
        return rows, nnz

    def level(self, l):
        d = _LevelDesc()
        _check(self.lib.giamg_level_describe(self._h, l, ctypes.byref(d)))
        return {"kind": LEVEL_KIND[d.kind], "order": d.order, "coarsest": bool(d.coarsest),
                "rows": d.rows, "nnz_A": d.nnz_A, "nnz_P": d.nnz_P, "nnz_R": d.nnz_R,
                "nnz_AP": d.nnz_AP, "lam_hat": d.lam_hat, "staged_nnz_A": d.staged_nnz_A,
                "runs_A": d.runs_A, "groups_A": d.groups_A, "group_entries_A": d.group_entries_A,
                "lean_A": bool(d.lean_A), "device_assembly": bool(d.device_assembly)}

    def level_csr(self, l, which="A"):
        d = self.level(l)
        if which == "A":
            nr, nnz = d["rows"], d["nnz_A"]
        elif which == "P":
            nr, nnz = d["rows"], d["nnz_P"]
        elif which == "AP":
            nr, nnz = d["rows"], d["nnz_AP"]
        else:
            nr, nnz = self.level(l + 1)["rows"], d["nnz_R"]
        rp = np.zeros(nr + 1, dtype=np.int64)
        ci = np.zeros(nnz, dtype=np.int32)
        val = np.zeros(nnz, dtype=np.float64)
        _check(self.lib.giamg_level_csr(self._h, l, MAT[which], _ptr(rp), _ptr(ci), _ptr(val)))
        return rp, ci, val

    def level_l2g(self, l):
        d = self.level(l)
        out = np.zeros((self.n_elem, (d["order"] + 1) ** 3), dtype=np.int32)
        _check(self.lib.giamg_level_l2g(self._h, l, _ptr(out)))
        return out

    def level_aggregates(self, l):
        out = np.zeros(self.level(l)["rows"], dtype=np.int32)
        _check(self.lib.giamg_level_aggregates(self._h, l, _ptr(out)))
        return out

    def constrained(self):
        out = np.zeros(self.n_nodes, dtype=np.uint8)
        _check(self.lib.giamg_constrained(self._h, _ptr(out)))
        return out.astype(bool)

    def apply(self, op, level, a, b=None, out=None, fp32=False):
        """One V-cycle step on device vectors of the level they live on
        (float64, or float32 with fp32=True): restrict reads level `level`
        and writes level + 1, prolong_add reads level + 1 and updates level
        `level`; b only for the residual."""
        import torch
        code = OP[op] | (OP_FP32 if fp32 else 0)
        nl = self.num_levels()
        if not 0 <= level < nl:
            raise ValueError(f"level {level} out of range (hierarchy of {nl} levels)")
        if op in ("restrict", "prolong_add") and level + 1 >= nl:
            raise ValueError(f"{op} needs a coarser level below level {level}")
        rows = self.level(level)["rows"]
        rows_c = self.level(level + 1)["rows"] if op in ("restrict", "prolong_add") else rows
        n_a = rows_c if op == "prolong_add" else rows
        n_out = rows_c if op == "restrict" else rows
        dt = torch.float32 if fp32 else torch.float64
        if out is None:
            raise ValueError("out is required")
        if op == "residual" and b is None:
            raise ValueError("the residual needs b (the iterate x)")
        if op != "residual" and b is not None:
            raise ValueError(f"{op} takes no b")
        specs = [(a, dt, (n_a,), "a"), (out, dt, (n_out,), "out")]
        if op == "residual":
            specs.append((b, dt, (rows,), "b"))
        ptrs = _devs(*specs)
        ap, op_ = ptrs[0], ptrs[1]
        bp = ptrs[2] if op == "residual" else ctypes.c_void_p()
        _check(self.lib.giamg_apply(self._h, code, level, ap, bp, op_))
        return out

    def quadrature_points(self):
        nq = self.p + 2
        xq = np.zeros((self.n_elem, nq ** 3, 3))
        _check(self.lib.giamg_quadrature_points(self._h, _ptr(xq)))
        return xq

    def load_vector(self, fq):
        fq = np.ascontiguousarray(fq, dtype=np.float64)
        b = np.zeros(self.n_nodes)
        _check(self.lib.giamg_load_vector(self._h, _ptr(fq), _ptr(b)))
        return b

    def time_kernel(self, kernel, level=0, reps=20, fp32=False):
        """Mean duration (ms) and algorithmic bytes of one launch."""
        ms, by = np.zeros(1), np.zeros(1)
        code = KERNEL[kernel] | (OP_FP32 if fp32 else 0)
        _check(self.lib.giamg_time_kernel(self._h, code, level, reps, _ptr(ms), _ptr(by)))
        return float(ms[0]), float(by[0])

    def profile(self, on=True, fine_step_only=False):
        """Profile the following solves: every phase (the breakdown), or
        only the launches of the fine Chebyshev step (fine_step_only)."""
        level = 0 if not on else (2 if fine_step_only else 1)
        _check(self.lib.giamg_profile_enable(self._h, level))

    def profile_read(self, reset=True):
        """{phase: (ms summed, intervals)} plus solves and iterations."""
        pr = _Profile()
        _check(self.lib.giamg_profile_read(self._h, ctypes.byref(pr), 1 if reset else 0))
        out = {name: (pr.ms[i], pr.count[i]) for i, name in enumerate(PHASES)}
        out["solves"] = pr.solves
        out["iterations"] = pr.iterations
        return out

    def setup_times(self):
        ms = np.zeros(7)
        _check(self.lib.giamg_setup_times(self._h, _ptr(ms)))
        keys = ["assembly", "p_transfer", "aggregation", "galerkin", "coarsest", "smoother", "total"]
        return dict(zip(keys, ms.tolist()))


def read_bandwidth(nbytes=1 << 30, reps=10):
    """Median GB/s of the library's streaming read kernel over reps reads of
    a buffer of nbytes on the current device."""
    g = np.zeros(1)
    _check(library().giamg_read_bandwidth(int(nbytes), int(reps), _ptr(g)))
    return float(g[0])


# ---- host-side setup steps (no GPU) ---------------------------------------
def _take_hcsr(h):
    lib = library()
    rows, cols, nnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    try:
        _check(lib.giamg_hcsr_size(h, ctypes.byref(rows), ctypes.byref(cols), ctypes.byref(nnz)))
        rp = np.zeros(rows.value + 1, dtype=np.int64)
        ci = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value, dtype=np.float64)
        _check(lib.giamg_hcsr_copy(h, _ptr(rp), _ptr(ci), _ptr(val)))
    finally:
        lib.giamg_hcsr_free(h)
    return rp, ci, val, (rows.value, cols.value)


def host_boundary(l2g, p, n_nodes, basis="nodal"):
    l2g = np.ascontiguousarray(l2g, dtype=np.int32)
    mask = np.zeros(n_nodes, dtype=np.uint8)
    _check(library().giamg_host_boundary(_ptr(l2g), l2g.shape[0], p, n_nodes, BASIS[basis],
                                         _ptr(mask)))
    return mask.astype(bool)


def host_assemble(coords, l2g, p, lam, bc="dirichlet", pin_node=0, basis="nodal"):
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    l2g = np.ascontiguousarray(l2g, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(library().giamg_host_assemble(_ptr(coords), coords.shape[0], _ptr(l2g), l2g.shape[0],
                                         p, float(lam), BC[bc], pin_node, BASIS[basis],
                                         ctypes.byref(h)))
    return _take_hcsr(h)


def host_p_transfer(l2g, p, q, n_fine, free_mask, basis="nodal"):
    l2g = np.ascontiguousarray(l2g, dtype=np.int32)
    fm = np.ascontiguousarray(free_mask, dtype=np.uint8)
    nxt = np.zeros((l2g.shape[0], (q + 1) ** 3), dtype=np.int32)
    nc = ctypes.c_int64()
    h = ctypes.c_void_p()
    _check(library().giamg_host_p_transfer(_ptr(l2g), l2g.shape[0], p, q, n_fine, _ptr(fm),
                                           BASIS[basis], _ptr(nxt), ctypes.byref(nc),
                                           ctypes.byref(h)))
    return nxt, nc.value, _take_hcsr(h)


def host_aggregate(rp, ci, val, seed=0, theta=0.0):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    n = rp.size - 1
    agg = np.zeros(n, dtype=np.int32)
    na = ctypes.c_int64()
    h = ctypes.c_void_p()
    _check(library().giamg_host_aggregate(_ptr(rp), _ptr(ci), _ptr(val), n, seed, float(theta),
                                          _ptr(agg), ctypes.byref(na), ctypes.byref(h)))
    return agg, na.value, _take_hcsr(h)


def host_coarse_inverse(A):
    """Dense inverse of a symmetric positive definite matrix as the setup
    forms it for the coarsest level (host float64 [n][n])."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    inv = np.empty_like(A)
    _check(library().giamg_host_coarse_inverse(_ptr(A), A.shape[0], _ptr(inv)))
    return inv


# ---- continuous batching ---------------------------------------------------
def _info(i):
    return SolveInfo(i.iters, i.status, i.relres, i.true_relres, i.solve_ms, i.bytes)


class Session:
    """Slots of one solver that right-hand sides join and leave between steps."""

    def __init__(self, solver: Solver, slots: int, tol: float = 1e-10):
        self.lib = library()
        self.solver = solver
        self.slots = slots
        self._s = ctypes.c_void_p()
        _check(self.lib.giamg_session_create(solver._h, slots, float(tol), ctypes.byref(self._s)))
        self._keep = {}

    def admit(self, slots, bs):
        """Start right-hand sides bs[i] (float64 device tensors of n_nodes
        entries) in slots[i]."""
        import torch
        if len(slots) != len(bs):
            raise ValueError("slots and bs must have the same length")
        for s_ in slots:
            if not 0 <= int(s_) < self.slots:
                raise ValueError(f"slot {s_} out of range [0, {self.slots})")
        n = (self.solver.n_nodes,)
        devs = _devs(*[(b, torch.float64, n, f"bs[{i}]") for i, b in enumerate(bs)])
        ptrs = (ctypes.c_void_p * len(bs))(*[d.value for d in devs])
        arr = (ctypes.c_int32 * len(slots))(*slots)
        for s_, b in zip(slots, bs):
            self._keep[s_] = b          # the kernels read b asynchronously
        _check(self.lib.giamg_session_admit(self._s, len(slots), arr, ptrs))

    def step(self, iters):
        _check(self.lib.giamg_session_step(self._s, iters))

    def poll(self):
        running = np.zeros(self.slots, dtype=np.int32)
        infos = (_Info * self.slots)()
        _check(self.lib.giamg_session_poll(self._s, _ptr(running), infos))
        return running.astype(bool), [_info(i) for i in infos]

    def retire(self, slot, out):
        import torch
        if not 0 <= int(slot) < self.slots:
            raise ValueError(f"slot {slot} out of range [0, {self.slots})")
        op_, = _devs((out, torch.float64, (self.solver.n_nodes,), "out"))
        _check(self.lib.giamg_session_retire(self._s, slot, op_))
        self._keep.pop(slot, None)
        return out

    def close(self):
        if self._s:
            self.lib.giamg_session_free(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request loop with continuous batching, device hierarchy cache and HBM
    budget (runs on a background thread inside the library)."""

    def __init__(self, hbm_budget, slots=8, chunk=2, tol=1e-10, hold_ms=0):
        self.lib = library()
        o = _ServerOpts(int(hbm_budget), int(slots), int(chunk), float(tol), int(hold_ms), 0)
        self._s = ctypes.c_void_p()
        _check(self.lib.giamg_server_create(ctypes.byref(o), ctypes.byref(self._s)))
        self._sizes = []
        self._out = {}

    def add_problem(self, coords, l2g, p, lam, opts: Options = None):
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        l2g = np.ascontiguousarray(l2g, dtype=np.int32)
        pid = ctypes.c_int32()
        co = (opts or Options())._c()
        _check(self.lib.giamg_server_add_problem(self._s, _ptr(coords), coords.shape[0], _ptr(l2g),
                                                 l2g.shape[0], int(p), float(lam), ctypes.byref(co),
                                                 ctypes.byref(pid)))
        self._sizes.append(coords.shape[0])
        return pid.value

    def submit(self, problem, b):
        if not 0 <= int(problem) < len(self._sizes):
            raise ValueError(f"unknown problem {problem}")
        b = np.ascontiguousarray(b, dtype=np.float64)
        if b.ndim != 1 or b.size != self._sizes[problem]:
            raise ValueError(f"b: expected {self._sizes[problem]} entries, got shape {b.shape}")
        x = np.zeros_like(b)
        rid = ctypes.c_int64()
        _check(self.lib.giamg_server_submit(self._s, problem, _ptr(b), _ptr(x), ctypes.byref(rid)))
        self._out[rid.value] = x
        return rid.value

    def wait(self, request):
        info = _Info()
        lat = ctypes.c_double()
        rc = self.lib.giamg_server_wait(self._s, request, ctypes.byref(info), ctypes.byref(lat))
        x = self._out.pop(request)
        if rc < 0:
            raise GiamgError(rc, library().giamg_last_error().decode())
        return x, _info(info), lat.value

    def stats(self):
        st = _ServerStats()
        _check(self.lib.giamg_server_stats(self._s, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_ if f != "pad"}

    def close(self):
        if self._s:
            self.lib.giamg_server_free(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
