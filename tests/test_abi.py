"""The C-ABI library loads and exports every entry point include/giamg.h
declares (no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "giamg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(giamg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("giamg_setup", "giamg_solve", "giamg_solve_batch", "giamg_free",
                     "giamg_last_error", "giamg_apply"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2512_15121_amd import giamg
    lib = ctypes.CDLL(giamg.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_2512_15121_amd import giamg
    assert set(_declared()) == set(giamg._SIGNATURES)


def test_errors_without_device_work():
    from paper_2512_15121_amd import giamg
    import numpy as np
    lib = giamg.library()
    h = ctypes.c_void_p()
    # p out of range is rejected before any device call
    coords = np.zeros((8, 3))
    l2g = np.arange(8, dtype=np.int32)[None, :]
    rc = lib.giamg_setup(giamg._ptr(coords), 8, giamg._ptr(l2g), 1, 11, 1.0, None, None,
                         ctypes.byref(h))
    assert rc == giamg.EINVAL and b"order" in lib.giamg_last_error()
    rc = lib.giamg_setup(giamg._ptr(coords), 8, giamg._ptr(l2g), 1, 1, -1.0, None, None,
                         ctypes.byref(h))
    assert rc == giamg.EINVAL and b"lambda" in lib.giamg_last_error()
    bad = l2g.copy()
    bad[0, 3] = 99
    rc = lib.giamg_setup(giamg._ptr(coords), 8, giamg._ptr(bad), 1, 1, 1.0, None, None,
                         ctypes.byref(h))
    assert rc == giamg.EINVAL and b"range" in lib.giamg_last_error()
    assert not h.value
    lib.giamg_free(None)


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes mirror has the C struct's size and field offsets, as gcc
    lays out include/giamg.h."""
    import shutil
    import subprocess
    from paper_2512_15121_amd import giamg
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    mirrors = {"giamg_opts": giamg._Opts, "giamg_info": giamg._Info, "giamg_profile": giamg._Profile,
               "giamg_level_desc": giamg._LevelDesc, "giamg_server_opts": giamg._ServerOpts,
               "giamg_server_statistics": giamg._ServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "giamg.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, py in mirrors.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, f"{cname}.{field}"


def test_option_constants_match_header():
    from paper_2512_15121_amd import giamg
    text = open(os.path.join(ROOT, "include", "giamg.h")).read()
    defs = {m.group(1): int(m.group(2))
            for m in re.finditer(r"#define\s+(GIAMG_\w+)\s+\(?(-?\d+)\)?", text)}
    for i, name in enumerate(giamg.PHASES):
        assert defs["GIAMG_PHASE_" + name.upper()] == i, name
    assert defs["GIAMG_PHASE_COUNT"] == len(giamg.PHASES)
    tables = {"GIAMG_BATCH_": giamg.BATCH_KERNEL, "GIAMG_BASIS_": giamg.BASIS,
              "GIAMG_BC_": giamg.BC, "GIAMG_PREC_": giamg.PRECISION,
              "GIAMG_SMOOTHER_": giamg.SMOOTHER, "GIAMG_PRECOND_": giamg.PRECONDITIONER,
              "GIAMG_KERNEL_": giamg.KERNEL, "GIAMG_ASSEMBLY_": giamg.ASSEMBLY}
    for prefix, table in tables.items():
        for name, value in table.items():
            assert defs[prefix + name.upper()] == value, prefix + name


def test_unknown_batch_kernel_is_rejected_before_device_work():
    from paper_2512_15121_amd import giamg
    import numpy as np
    lib = giamg.library()
    o = giamg._Opts()
    lib.giamg_default_opts(ctypes.byref(o))
    assert o.batch_kernel == giamg.BATCH_KERNEL["auto"]
    o.batch_kernel = 7
    coords = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], dtype=np.float64)
    l2g = np.arange(8, dtype=np.int32)[None, :]
    h = ctypes.c_void_p()
    rc = lib.giamg_setup(giamg._ptr(coords), 8, giamg._ptr(l2g), 1, 1, 1.0, ctypes.byref(o), None,
                         ctypes.byref(h))
    assert rc == giamg.EINVAL and b"batch_kernel" in lib.giamg_last_error()
    assert not h.value


def test_row_groups_option_default_and_validation():
    from paper_2512_15121_amd import giamg
    import numpy as np
    lib = giamg.library()
    o = giamg._Opts()
    lib.giamg_default_opts(ctypes.byref(o))
    assert o.row_groups == 0
    o.row_groups = 2
    coords = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], dtype=np.float64)
    l2g = np.arange(8, dtype=np.int32)[None, :]
    h = ctypes.c_void_p()
    rc = lib.giamg_setup(giamg._ptr(coords), 8, giamg._ptr(l2g), 1, 1, 1.0, ctypes.byref(o), None,
                         ctypes.byref(h))
    assert rc == giamg.EINVAL and b"row_groups" in lib.giamg_last_error()
    assert not h.value


def test_lean_threshold_default_and_validation():
    from paper_2512_15121_amd import giamg
    import numpy as np
    lib = giamg.library()
    o = giamg._Opts()
    lib.giamg_default_opts(ctypes.byref(o))
    assert o.lean_max_nnz == 2000000 and giamg.Options().lean_max_nnz == 2000000
    o.lean_max_nnz = -1
    coords = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], dtype=np.float64)
    l2g = np.arange(8, dtype=np.int32)[None, :]
    h = ctypes.c_void_p()
    rc = lib.giamg_setup(giamg._ptr(coords), 8, giamg._ptr(l2g), 1, 1, 1.0, ctypes.byref(o), None,
                         ctypes.byref(h))
    assert rc == giamg.EINVAL and b"lean_max_nnz" in lib.giamg_last_error()
    assert not h.value


def test_set_allocator_validation_without_device_work():
    from paper_2512_15121_amd import giamg
    lib = giamg.library()
    rc = lib.giamg_set_allocator(giamg.ALLOC_FN(lambda n, s, c: None), giamg.RELEASE_FN(), None)
    assert rc == giamg.EINVAL and b"both" in lib.giamg_last_error()
    giamg.set_allocator(lambda n, s: 0, lambda p: None)   # registering touches no device
    giamg.set_allocator()


def test_host_stages_reject_malformed_input():
    """The host-stage entry points check sizes and the CSR row pointer before
    reading the arrays they describe."""
    from paper_2512_15121_amd import giamg
    import numpy as np
    lib = giamg.library()
    out = ctypes.c_void_p()
    n_agg = ctypes.c_int64()
    agg = np.zeros(2, dtype=np.int32)
    col = np.array([0, 1, 0, 1], dtype=np.int32)
    val = np.ones(4)
    for rp, word in (([1, 2, 4], b"row_ptr[0]"), ([0, 3, 2], b"non-decreasing")):
        rp = np.array(rp, dtype=np.int64)
        rc = lib.giamg_host_aggregate(giamg._ptr(rp), giamg._ptr(col), giamg._ptr(val), 2, 0, 0.0,
                                      giamg._ptr(agg), ctypes.byref(n_agg), ctypes.byref(out))
        assert rc == giamg.EINVAL and word in lib.giamg_last_error()
        assert not out.value
    l2g = np.arange(27, dtype=np.int32)
    free = np.ones(27, dtype=np.uint8)
    nxt = np.zeros(8, dtype=np.int32)
    n_c = ctypes.c_int64()
    for n_elem, p, n_fine in ((0, 2, 27), (1, 2, 0), (1, 11, 27)):
        rc = lib.giamg_host_p_transfer(giamg._ptr(l2g), n_elem, p, 1, n_fine, giamg._ptr(free),
                                       giamg.BASIS["nodal"], giamg._ptr(nxt), ctypes.byref(n_c),
                                       ctypes.byref(out))
        assert rc == giamg.EINVAL, (n_elem, p, n_fine)
        assert not out.value


def test_theta_and_hierarchy_info_validation_without_device_work():
    """theta defaults to 0 and is checked in setup and the host aggregation
    stage; giamg_hierarchy_info rejects a null handle."""
    from paper_2512_15121_amd import giamg
    import numpy as np
    lib = giamg.library()
    o = giamg._Opts()
    lib.giamg_default_opts(ctypes.byref(o))
    assert o.theta == 0.0 and giamg.Options().theta == 0.0
    o.theta = 1.5
    coords = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], dtype=np.float64)
    l2g = np.arange(8, dtype=np.int32)[None, :]
    h = ctypes.c_void_p()
    rc = lib.giamg_setup(giamg._ptr(coords), 8, giamg._ptr(l2g), 1, 1, 1.0, ctypes.byref(o), None,
                         ctypes.byref(h))
    assert rc == giamg.EINVAL and b"theta" in lib.giamg_last_error()
    assert not h.value
    rp = np.array([0, 2, 4], dtype=np.int64)
    col = np.array([0, 1, 0, 1], dtype=np.int32)
    val = np.array([2.0, -1.0, -1.0, 2.0])
    agg = np.zeros(2, dtype=np.int32)
    n_agg = ctypes.c_int64()
    out = ctypes.c_void_p()
    rc = lib.giamg_host_aggregate(giamg._ptr(rp), giamg._ptr(col), giamg._ptr(val), 2, 0, -0.1,
                                  giamg._ptr(agg), ctypes.byref(n_agg), ctypes.byref(out))
    assert rc == giamg.EINVAL and b"theta" in lib.giamg_last_error() and not out.value
    nl = ctypes.c_int32(-7)
    rc = lib.giamg_hierarchy_info(None, ctypes.byref(nl), None, None, 0)
    assert rc == giamg.EINVAL and nl.value == -7
    assert lib.giamg_profile_enable(None, 1) == giamg.EINVAL
    g = np.zeros(1)
    assert lib.giamg_read_bandwidth(1024, 3, giamg._ptr(g)) == giamg.EINVAL
    assert b"1 MiB" in lib.giamg_last_error()
    assert lib.giamg_read_bandwidth(1 << 20, 0, giamg._ptr(g)) == giamg.EINVAL


def test_server_options_are_checked_before_device_work():
    """Out-of-range server options (a negative or over-long admission hold,
    no slots) are rejected before the library touches a device."""
    from paper_2512_15121_amd import giamg
    lib = giamg.library()
    for kw in ({"hold_ms": -1}, {"hold_ms": 60001}, {"slots": 0}, {"chunk": 0}):
        f = dict(hbm_budget=1 << 30, slots=4, chunk=2, tol=1e-10, hold_ms=0, pad=0)
        f.update(kw)
        o = giamg._ServerOpts(**f)
        s = ctypes.c_void_p()
        assert lib.giamg_server_create(ctypes.byref(o), ctypes.byref(s)) == giamg.EINVAL, kw
        assert b"server options" in lib.giamg_last_error()
        assert not s.value
