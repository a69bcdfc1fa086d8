"""The C-ABI library loads and exports every entry point include/amg.h declares
(host-only checks; no GPU work is launched)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "amg.h")
LIB = os.path.join(ROOT, "paper_1302_2547_amd", "libamg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amg_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libamg.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("amg_setup", "amg_solve", "amg_free", "amg_export_level", "amg_default_options"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_only_paths(lib):
    from paper_1302_2547_amd import amg
    o = amg.default_options()
    assert o.coarsest_size == 64 and o.max_levels == 40 and o.kcycle_inner == 2
    assert abs(o.stall_ratio - 0.9) < 1e-15 and o.max_iters == 200 and o.precision == amg.AMG_PREC_FP64
    assert o.smoother == amg.AMG_SMOOTHER_L1 and o.jacobi_weight == 2.0 / 3.0 and o.autotune == 1
    assert amg.amg_status_string(amg.AMG_ERR_BREAKDOWN) == b"AMG_ERR_BREAKDOWN"
    # argument errors are reported before any device work
    out = ctypes.c_void_p(123)
    assert amg.amg_setup(None, None, ctypes.byref(out)) == amg.AMG_ERR_INVALID_ARGUMENT
    assert out.value is None
    bad = amg.amg_csr(0, 0, None, None, None)
    assert amg.amg_setup(ctypes.byref(bad), None, ctypes.byref(out)) == amg.AMG_ERR_INVALID_ARGUMENT
    assert amg.amg_solve(None, None, None, 1e-8, None) == amg.AMG_ERR_INVALID_ARGUMENT
    amg.amg_free(None)
    n = ctypes.c_int32()
    assert amg.amg_num_levels(None, ctypes.byref(n)) == amg.AMG_ERR_INVALID_ARGUMENT
    slots = ctypes.c_int64()
    assert amg.amg_level_slots(None, 0, ctypes.byref(slots)) == amg.AMG_ERR_INVALID_ARGUMENT


def test_host_arrays_are_rejected(lib):
    """Entry points that take device arrays refuse pageable host memory (an error
    status, never a kernel writing through a host address)."""
    import numpy as np
    from paper_1302_2547_amd import amg
    host = np.zeros(64, np.float64)
    hi = np.zeros(65, np.int32)
    assert amg.amg_uniform_rhs(64, 1, host.ctypes.data, None) == amg.AMG_ERR_INVALID_ARGUMENT
    dims = (ctypes.c_int32 * 3)(4, 4, 1)
    assert amg.amg_grid_laplacian(2, dims, 0.1, 1, hi.ctypes.data, hi.ctypes.data, host.ctypes.data,
                                  None) == amg.AMG_ERR_INVALID_ARGUMENT
    csr = amg.amg_csr(8, 8, hi.ctypes.data, hi.ctypes.data, host.ctypes.data)
    out = ctypes.c_void_p()
    assert amg.amg_setup(ctypes.byref(csr), None, ctypes.byref(out)) == amg.AMG_ERR_INVALID_ARGUMENT
    assert amg.amg_grid_laplacian_nnz(2, dims) == 16 + 2 * 2 * 4 * 3


def test_options_struct_matches_header():
    from paper_1302_2547_amd import amg
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    block = text[text.index("int32_t coarsest_size"):]
    block = block[:block.index("} amg_options;")]
    fields = re.findall(r"\b([a-z_]+);", block)
    assert fields == [f for f, _ in amg.amg_options._fields_]


def test_group_job_struct_matches_header():
    from paper_1302_2547_amd import amg
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    block = text[text.index("amg_hierarchy *h;"):]
    block = block[:block.index("} amg_group_job;")]
    fields = re.findall(r"\b([a-z_]+);", block)
    assert fields == [f for f, _ in amg.amg_group_job._fields_]
    assert ctypes.sizeof(amg.amg_group_job) == 32


def test_group_argument_errors(lib):
    """The grouped entry points check their arguments before any device work."""
    from paper_1302_2547_amd import amg
    st = (ctypes.c_int32 * 2)()
    jobs = (amg.amg_group_job * 2)()
    assert amg.amg_solve_group(0, None, 1e-8, None, None, None) == amg.AMG_OK
    assert amg.amg_solve_group(-1, jobs, 1e-8, None, st, None) == amg.AMG_ERR_INVALID_ARGUMENT
    assert amg.amg_solve_group(1, None, 1e-8, None, st, None) == amg.AMG_ERR_INVALID_ARGUMENT
    assert amg.amg_solve_group(1, jobs, 1e-8, None, None, None) == amg.AMG_ERR_INVALID_ARGUMENT
    assert amg.amg_solve_group(1, jobs, 1e-8, None, st, None) == amg.AMG_ERR_INVALID_ARGUMENT  # h NULL
    assert amg.amg_solve_group(1, jobs, 0.0, None, st, None) == amg.AMG_ERR_INVALID_ARGUMENT
    assert amg.amg_kcycle_group(1, jobs, None, st) == amg.AMG_ERR_INVALID_ARGUMENT
    assert amg.amg_kcycle_group(0, None, None, None) == amg.AMG_OK
