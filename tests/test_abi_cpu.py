"""Host-side checks of the C ABI: the library loads without a GPU and
exports every function that include/mg.h declares; option defaults."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("mg_create_hierarchy", "mg_solve", "mg_residual_norm", "mg_destroy_hierarchy", "mg_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1104_1703_amd import mg
    if not os.path.exists(mg.LIB_PATH):
        pytest.skip("libmg.so not built")
    lib = mg.load_library()
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(n for n, _, _ in mg.SYMBOLS) == _declared()


def test_default_options_follow_the_paper():
    from paper_1104_1703_amd import mg
    if not os.path.exists(mg.LIB_PATH):
        pytest.skip("libmg.so not built")
    o = mg.default_options()
    assert (o.n_pre, o.n_post, o.n_cycles) == (2, 2, 1)      # Sec. 2: N_pre = N_post = 2, V-cycles
    assert o.eta == 0.5 and o.first_order_hold == 10          # Sec. 4 switch
    assert o.n_coarse_sweeps == 32 and o.min_coarse_dim == 4
    assert o.bc_order == mg.MG_BC_AUTO and o.precision == mg.MG_FP64


def test_status_strings():
    from paper_1104_1703_amd import mg
    if not os.path.exists(mg.LIB_PATH):
        pytest.skip("libmg.so not built")
    lib = mg.load_library()
    for s in (0, 1, -1, -2, -3, -4, -5):
        assert lib.mg_status_string(s)
    assert lib.mg_status_string(99) == b"unknown status"


def test_create_rejects_null_arguments_without_gpu():
    """Argument checks happen before any device call."""
    import ctypes as C
    from paper_1104_1703_amd import mg
    if not os.path.exists(mg.LIB_PATH):
        pytest.skip("libmg.so not built")
    lib = mg.load_library()
    out = C.c_void_p()
    assert lib.mg_create_hierarchy(None, 8, 8, 8, 0.1, None, None, C.byref(out)) == mg.MG_ERR_ARG
    assert lib.mg_create_hierarchy(C.c_void_p(1), 8, 8, 8, -1.0, None, None, C.byref(out)) == mg.MG_ERR_ARG
    assert lib.mg_solve(None, None, None, None, 1e-10, None) == mg.MG_ERR_ARG
    assert lib.mg_batch_validate(None, None, 0) == -1
    assert lib.mg_level_item_depth(None, 0, 2) == -1
    ms, n = C.c_double(0.0), C.c_int32(0)
    assert lib.mg_kernel_timing(None, 1) == mg.MG_ERR_ARG
    assert lib.mg_kernel_timing_read(None, C.byref(ms), C.byref(n)) == mg.MG_ERR_ARG
