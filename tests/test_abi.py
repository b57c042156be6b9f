"""Host-side checks of the C ABI (no GPU needed): librsvd.so loads, exports
every function include/rsvd.h declares, and rejects bad arguments before any
device call."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "rsvd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_1906_12085_amd as pk
    if not os.path.exists(pk.LIB_PATH):
        pytest.fail("librsvd.so is not built (run __graft_entry__.build())")
    return pk.load_library()


def test_header_parses_all_entry_points():
    names = declared_functions()
    assert "rsvd_solve" in names and "gram_eig_solve" in names and len(names) >= 14


def test_every_declared_symbol_is_exported(lib):
    import paper_1906_12085_amd as pk
    names = declared_functions()
    for name in names:
        assert hasattr(lib, name), f"{name} declared in rsvd.h but not exported"
    assert sorted(pk.EXPORTS) == names


def test_status_strings(lib):
    import paper_1906_12085_amd as pk
    for code, name in pk.STATUS.items():
        assert pk.rsvd_status_string(code) == name
    assert pk.rsvd_status_string(12345) == "RSVD_UNKNOWN_STATUS"


def test_plan_create_validates_before_device_calls(lib):
    h = ctypes.c_void_p()
    f = lib.rsvd_plan_create
    assert f(None, 100, 10, 8, 0, 0, 0, None) == -1                       # NULL out-pointer
    assert f(ctypes.byref(h), 100, 10, 8, 7, 0, 0, None) == -1            # bad dtype
    assert f(ctypes.byref(h), 100, 10, 0, 0, 0, 0, None) == -1            # l_max < 1
    assert f(ctypes.byref(h), 5, 10, 8, 0, 0, 0, None) == -2              # m_max < n_max
    assert f(ctypes.byref(h), 100, 0, 8, 0, 0, 0, None) == -2             # n_max < 1
    assert f(ctypes.byref(h), 1000, 200, 193, 1, 0, 0, None) == -2        # l_max above 192
    assert f(ctypes.byref(h), 5000, 2000, 32, 1, 1, 0, None) == -2        # A^T A route n_max above 1024
    assert f(ctypes.byref(h), 5000, 200, 32, 2, 1, 0, None) == -1         # bf16 plan: no A^T A route
    assert f(ctypes.byref(h), 5000, 200, 32, 3, 1, 0, None) == -1         # fp8 plan: no A^T A route
    assert f(ctypes.byref(h), 5000, 200, 32, 4, 0, 0, None) == -1         # unknown dtype
    b = lib.rsvd_batch_create
    assert b(None, 2, 1000, 100, 16, 1, 0) == -1                          # batch NULL
    assert b(ctypes.byref(h), 0, 1000, 100, 16, 1, 0) == -1               # no slots
    assert b(ctypes.byref(h), 65, 1000, 100, 16, 1, 0) == -1              # too many slots
    assert b(ctypes.byref(h), 2, 1000, 100, 16, 4, 0) == -1               # unknown dtype
    sv = lib.rsvd_server_create
    assert sv(None, 2, 1000, 100, 16, 1, 0, 1 << 30, 0) == -1             # server NULL
    assert sv(ctypes.byref(h), 2, 1000, 100, 16, 1, 0, 0, 0) == -1        # no budget
    assert sv(ctypes.byref(h), 0, 1000, 100, 16, 1, 0, 1 << 30, 0) == -1  # no slots
    assert sv(ctypes.byref(h), 2, 1000, 100, 16, 1, 0, 1 << 30, 4) == -1  # unknown flag
    assert sv(ctypes.byref(h), 2, 5000, 2000, 16, 1, 0, 1 << 30, 1) == -2  # fallback n_max > 1024
    assert h.value is None


def test_solvers_reject_null_plan(lib):
    a = ctypes.c_void_p(16)
    assert lib.rsvd_solve(None, a, 100, 10, 10, None, 2, 2, 1, 0.9, a, 2, a, a, 2, a) == -1
    assert lib.rsvd_solve_omega(None, a, 100, 10, 10, None, 2, 2, 1, 0.9, None, a, 2, a, a, 2,
                                a) == -1
    assert lib.gram_eig_solve(None, a, 100, 10, 10, 0.9, 0, None, 0, a, a, 10, a) == -1
    assert lib.rsvd_gemm_nn(None, a, 10, 10, 10, a, 4, 4, a, 4, None, None) == -1
    assert lib.rsvd_plan_status(None) == -1
    assert lib.rsvd_plan_destroy(None) == 0
    assert lib.rsvd_gaussian_fill(1, 4, 4, None, None) == -1
    assert lib.rsvd_plan_kernel_times(None, 1, None, None, 0) == -1
    assert lib.rsvd_solve_bf16(None, a, None, 100, 16, 16, 4, 2, 1, 0.9, None, a, 4, a, a, 4, a) == -1
    assert lib.rsvd_quantize_bf16(None, a, 100, 16, 16, a, 16, a) == -1
    assert lib.rsvd_solve_fp8(None, a, None, 100, 16, 16, 4, 2, 1, 0.9, None, a, 4, a, a, 4, a) == -1
    assert lib.rsvd_quantize_fp8(None, a, 100, 16, 16, a, 16, a) == -1
    assert lib.rsvd_solve_krylov(None, a, 100, 10, 10, 2, 2, 1, 0.9, None, a, 2, a, a, 2, a) == -1
    assert lib.rsvd_solve_adaptive(None, a, 100, 10, 10, None, 2, 2, 1, 0.9, 4, a, 4, a, a, 4,
                                   a) == -1
    assert lib.rsvd_batch_solve(None, None, 0, None) == -1
    assert lib.rsvd_batch_graph_create(None, None, 0, None, None) == -1
    assert lib.rsvd_batch_graph_launch(None, None) == -1
    assert lib.rsvd_batch_destroy(None) == 0
    assert lib.rsvd_batch_graph_destroy(None) == 0
    assert lib.rsvd_server_submit(None, None, None) == -1
    assert lib.rsvd_server_progress(None, None, 0, None, None, None) == -1
    assert lib.rsvd_server_destroy(None) == 0
    # grouped batches: null handles, negative counts and tables are argument
    # errors before any device call
    g = ctypes.c_void_p()
    assert lib.rsvd_batch_grouped_create(None, None, 0, None, 0, ctypes.byref(g)) == -1
    assert lib.rsvd_batch_grouped_create(a, None, 0, None, -1, ctypes.byref(g)) == -1
    assert lib.rsvd_batch_grouped_create(a, None, 0, None, 2, ctypes.byref(g)) == -1
    assert lib.rsvd_batch_grouped_launch(None, None) == -1
    assert lib.rsvd_batch_grouped_destroy(None) == 0
    assert lib.rsvd_batch_grouped_graph_create(None, ctypes.byref(g)) == -1
    nout = ctypes.c_int32()
    assert lib.rsvd_batch_grouped_tune(None, None, 0, None, 0, ctypes.byref(nout), None) == -1
    import paper_1906_12085_amd as pk
    tab = (pk.RsvdTuneEntry * 4)()
    assert lib.rsvd_batch_grouped_tune(a, None, -1, tab, 4, ctypes.byref(nout), None) == -1
    assert lib.rsvd_batch_grouped_tune(a, None, 0, tab, -1, ctypes.byref(nout), None) == -1
    assert lib.rsvd_batch_grouped_tune(a, None, 0, None, 4, ctypes.byref(nout), None) == -1


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_1906_12085_amd as pk
    saved = pk._lib
    try:
        pk._lib = None
        with pytest.raises(ImportError):
            pk.load_library(str(tmp_path / "missing.so"))
    finally:
        pk._lib = saved
