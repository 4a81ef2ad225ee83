"""The C ABI without a GPU: the library loads, exports every function that
include/spamm.h declares, and rejects bad arguments before touching HIP."""
import ctypes
import re

import pytest

import paper_1203_1692_amd as sp


def test_library_exports_every_declared_symbol():
    lib = sp.load()
    names = sp.header_functions()
    assert "spamm_build_tree" in names and "spamm_multiply" in names
    for name in names:
        assert hasattr(lib, name), name


def test_header_status_codes_match_binding():
    text = open(sp.HEADER).read()
    codes = dict((m[0], int(m[1])) for m in re.findall(r"#define (SPAMM_[A-Z_]+)\s+(-?\d+)", text))
    assert codes["SPAMM_OK"] == sp.SPAMM_OK
    assert codes["SPAMM_E_INVAL"] == sp.SPAMM_E_INVAL
    assert codes["SPAMM_E_NONFINITE"] == sp.SPAMM_E_NONFINITE
    assert codes["SPAMM_E_NOMEM"] == sp.SPAMM_E_NOMEM
    assert codes["SPAMM_E_HIP"] == sp.SPAMM_E_HIP
    assert codes["SPAMM_E_RANGE"] == sp.SPAMM_E_RANGE
    assert codes["SPAMM_E_MISMATCH"] == sp.SPAMM_E_MISMATCH
    assert codes["SPAMM_E_BUSY"] == sp.SPAMM_E_BUSY
    assert codes["SPAMM_PENDING"] == sp.SPAMM_PENDING


def test_header_precision_and_tree_flags_match_binding():
    text = open(sp.HEADER).read()
    defs = dict((m[0], int(m[1])) for m in
                re.findall(r"#define (SPAMM_(?:PREC|TREE)_[A-Z0-9_]+)\s+(\d+)u?", text))
    assert defs == {"SPAMM_PREC_FP32": sp.PREC_FP32, "SPAMM_PREC_SPLIT_BF16": sp.PREC_SPLIT_BF16,
                    "SPAMM_PREC_SPLIT_FP16": sp.PREC_SPLIT_FP16,
                    "SPAMM_PREC_SPLIT_BF16X3": sp.PREC_SPLIT_BF16X3,
                    "SPAMM_TREE_BF16": sp.TREE_BF16, "SPAMM_TREE_SUBNORMS": sp.TREE_SUBNORMS,
                    "SPAMM_TREE_FP16": sp.TREE_FP16}
    # tree flags are distinct bits
    flags = [v for k, v in defs.items() if k.startswith("SPAMM_TREE_")]
    assert all(f & (f - 1) == 0 for f in flags) and len(set(flags)) == len(flags)


def test_strerror_names_every_code():
    for code in (0, -1, -2, -3, -4, -5, -6, -7, 1):
        assert sp.strerror(code) != "unknown status"
    assert sp.strerror(-99) == "unknown status"


def test_argument_checks_before_any_device_call():
    lib = sp.load()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(4096)
    assert lib.spamm_build_tree(None, 64, 32, None, ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree(fake, 0, 32, None, ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree(fake, 64, 48, None, ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree(fake, 64, 128, None, ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree(fake, 64, 32, None, None) == sp.SPAMM_E_INVAL
    # more than 1024 leaves per dimension
    assert lib.spamm_build_tree(fake, 16 * 1024 + 1, 16, None, ctypes.byref(h)) == sp.SPAMM_E_RANGE
    assert b"tiers" in lib.spamm_last_error()
    assert lib.spamm_symbolic(None, None, 0.0, None, ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_numeric(None, None, None) == sp.SPAMM_E_INVAL
    assert lib.spamm_multiply(None, None, 1e-6, fake, None) == sp.SPAMM_E_INVAL
    assert lib.spamm_tree_info(None, None, None, None, None) == sp.SPAMM_E_INVAL
    assert lib.spamm_tree_free(None) == sp.SPAMM_OK
    assert lib.spamm_plan_free(None) == sp.SPAMM_OK
    opts = sp.Opts(1e-6, sp.PREC_FP32, 0.0, 0, 0.0)
    assert lib.spamm_multiply_noalloc(None, None, ctypes.byref(opts), fake,
                                      None) == sp.SPAMM_E_INVAL
    assert lib.spamm_multiply_noalloc(fake, fake, None, fake, None) == sp.SPAMM_E_INVAL
    assert lib.spamm_multiply_noalloc(fake, fake, ctypes.byref(opts), None,
                                      None) == sp.SPAMM_E_INVAL


def test_python_binding_rejects_cpu_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        sp.build_tree(torch.zeros(8, 8), 16)


def test_newer_entry_points_check_arguments_on_the_host():
    lib = sp.load()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(4096)
    dbl = ctypes.c_double
    # epsilon-sparsified build: flags, tolerance and the other operand's norm
    assert lib.spamm_build_tree_sparse(fake, 64, 32, 2, dbl(1e-6), dbl(0.0), None,
                                       ctypes.byref(h)) == sp.SPAMM_E_INVAL   # SUBNORMS
    assert lib.spamm_build_tree_sparse(fake, 64, 16, 1, dbl(1e-6), dbl(0.0), None,
                                       ctypes.byref(h)) == sp.SPAMM_E_INVAL   # BF16 at leaf 16
    for tau in (-1.0, float("nan"), float("inf"), 1e-200):
        assert lib.spamm_build_tree_sparse(fake, 64, 32, 0, dbl(tau), dbl(0.0), None,
                                           ctypes.byref(h)) == sp.SPAMM_E_INVAL
    for other in (-1.0, float("nan"), float("inf")):
        assert lib.spamm_build_tree_sparse(fake, 64, 32, 0, dbl(1e-6), dbl(other), None,
                                           ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree_sparse(None, 64, 32, 0, dbl(1e-6), dbl(0.0), None,
                                       ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree_sparse(fake, 64, 32, 0, dbl(1e-6), dbl(0.0), None,
                                       None) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree_sparse(fake, 16 * 1024 + 1, 16, 0, dbl(1e-6), dbl(0.0), None,
                                       ctypes.byref(h)) == sp.SPAMM_E_RANGE
    # sub-block norms only for 64 x 64 leaves; unknown flags; FP16 copies not
    # with BF16 ones, not for 16 x 16 leaves, not in a sparsified tree
    assert lib.spamm_build_tree_ex(fake, 64, 32, 2, None, ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree_ex(fake, 64, 64, 8, None, ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree_ex(fake, 64, 64, sp.TREE_FP16 | sp.TREE_BF16, None,
                                   ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree_ex(fake, 64, 16, sp.TREE_FP16, None,
                                   ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree_sparse(fake, 64, 32, sp.TREE_FP16, dbl(1e-6), dbl(0.0), None,
                                       ctypes.byref(h)) == sp.SPAMM_E_INVAL
    # tree of a product's output: NULL C, plan or out
    assert lib.spamm_build_tree_output(None, fake, 0, None, ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree_output(fake, None, 0, None, ctypes.byref(h)) == sp.SPAMM_E_INVAL
    assert lib.spamm_build_tree_output(fake, fake, 0, None, None) == sp.SPAMM_E_INVAL
    # NULL handles
    assert lib.spamm_tree_storage(None, None, None, None) == sp.SPAMM_E_INVAL
    assert lib.spamm_tree_matrix16(None, 0, None, 0, None, 0) == sp.SPAMM_E_INVAL
    cnt = ctypes.c_size_t()
    assert lib.spamm_plan_subtasks(None, None, 0, ctypes.byref(cnt)) == sp.SPAMM_E_INVAL
    assert lib.spamm_plan_stats(None, None) == sp.SPAMM_E_INVAL
    assert lib.spamm_plan_tasks(None, None, 0, ctypes.byref(cnt)) == sp.SPAMM_E_INVAL
    assert h.value is None
