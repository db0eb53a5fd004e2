"""The C-ABI library loads without a GPU and exports every function include/*.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(tdbem_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_binding_symbols():
    import paper_1503_07221_amd as tb
    assert declared_functions() == sorted(tb.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol():
    import paper_1503_07221_amd as tb
    if not os.path.exists(tb.LIB_PATH):
        pytest.skip("libtdbem.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(tb.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_null_context_is_rejected_without_a_device():
    """Calls on a NULL context fail with TDBEM_EINVAL before any HIP call."""
    import paper_1503_07221_amd as tb
    if not os.path.exists(tb.LIB_PATH):
        pytest.skip("libtdbem.so not built")
    lib = tb.load_library()
    assert lib.tdbem_assemble(None, 0, None) == -1
    assert lib.tdbem_matvec(None, None, None) == -1
    assert lib.tdbem_matvec_free(None, None, None, None) == -1
    assert lib.tdbem_set_time_grid(None, None, 2, 0, 0) == -1
    assert lib.tdbem_block_nnz(None, 0, 0, None) == -1
    assert lib.tdbem_get_block_coo(None, 0, 0, None, None, None, 0) == -1
    assert lib.tdbem_solve(None, None, None, None, None) == -1
    assert lib.tdbem_lp_init(None, 4, 0) == -1
    assert lib.tdbem_matvec_multi(None, 2, None, None) == -1
    assert lib.tdbem_potential_dl(None, None, 1, None, 1, None, None) == -1
    assert lib.tdbem_matvec_multi_tuning(None, None, None, None) == -1
    assert lib.tdbem_matvec_multi_set_variant(None, 0, None) == -1
    assert lib.tdbem_assemble_group(None, 2, 0, None) == -1
    assert lib.tdbem_solve_multi(None, 2, None, None, None, None) == -1
    assert lib.tdbem_lp_apply(None, None, None) == -1
    assert lib.tdbem_lp_gradient(None, None, None, None, None) == -1
    assert lib.tdbem_matvec_transpose(None, None, None) == -1
    assert lib.tdbem_lp_train(None, None, None, None) == -1
    assert lib.tdbem_lp_make_pairs(None, 1, 0, None, None) == -1
    assert lib.tdbem_assemble_tuning(None, None, None, None) == -1
    assert lib.tdbem_assemble_set_tiles(None, 0, None) == -1
    assert lib.tdbem_set_block_reuse(None, 1) == -1
    assert lib.tdbem_lp_train_pairs(None, None, None, None, 1, None, None, None) == -1
    assert lib.tdbem_lp_num_params(4) == 66112 and lib.tdbem_lp_num_params(0) == -1
    lib.tdbem_destroy(None)
    assert lib.tdbem_last_error(None) == b"null context"
    assert lib.tdbem_create(None, None) == -1


def test_create_rejects_options_it_cannot_meet():
    """tdbem_options: a deterministic flag other than 0/1, a regular rule other than the 7-point one
    and a table tolerance below what the tables reach are refused before any device call."""
    import ctypes
    import paper_1503_07221_amd as tb
    lib = tb.load_library()
    h = ctypes.c_void_p()
    for kw in ({"deterministic": 2}, {"quad_regular": 6}, {"psi_tol": 1e-14}, {"psi_tol": -1.0}, {"ss_order": 6}):
        opt = tb._Options(0, None, kw.get("ss_order", 4), kw.get("deterministic", 0), kw.get("quad_regular", 7),
                          kw.get("psi_tol", 0.0))
        assert lib.tdbem_create(ctypes.byref(h), ctypes.byref(opt)) == -1, kw


def test_package_does_not_import_the_oracle():
    """The product path never routes through the CPU oracle."""
    for root, _, files in os.walk(os.path.join(ROOT, "paper_1503_07221_amd")):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(root, f)).read()
                assert "oracle" not in txt.lower(), f
