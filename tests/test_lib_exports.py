"""The C-ABI library builds, loads and exports every symbol that include/lma.h
declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

import paper_1411_4510_amd as lma

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(name="lma.h"):
    src = open(os.path.join(ROOT, "include", name)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lma_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = header_functions()
    for n in ("lma_fit", "lma_predict", "lma_lml", "lma_free", "lma_last_error", "lma_failed_block"):
        assert n in names
    assert set(names) == set(lma.EXPORTS)
    assert set(header_functions("lma_ds.h")) == set(lma.DS_EXPORTS)


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(lma.LIB_PATH):
        pytest.fail("liblma.so not built (run paper_1411_4510_amd.build)")
    return ctypes.CDLL(lma.LIB_PATH)


def test_library_exports_every_declared_symbol(so):
    for name in header_functions() + header_functions("lma_ds.h"):
        assert hasattr(so, name), name


def test_version_and_error_without_gpu(so):
    so.lma_version.restype = ctypes.c_char_p
    assert so.lma_version().decode().startswith("lma-gfx950")
    so.lma_last_error.restype = ctypes.c_char_p
    # argument errors are detected on the host before any device call
    so.lma_fit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    so.lma_fit.restype = ctypes.c_int
    h = ctypes.c_void_p()
    assert so.lma_fit(None, None, ctypes.byref(h)) == lma.LMA_E_ARG
    assert "NULL" in so.lma_last_error().decode()


def test_binding_struct_matches_header_layout():
    # lma_problem: 5 int64, 6 pointers/doubles in order, then int32 x2 and int64
    assert ctypes.sizeof(lma._Problem) == 5 * 8 + 5 * 8 + 8 + 4 + 4 + 8


def test_profile_struct_matches_header_layout():
    # lma_profile: 6 doubles, 2 int64, 4 doubles, 2 int64
    assert ctypes.sizeof(lma.Profile) == 14 * 8
    names = [f for f, _ in lma.Profile._fields_]
    assert names[:8] == ["update_ms", "diag_ms", "trsm_ms", "other_ms", "update_alg_flops",
                         "update_alg_flops_f64", "update_launches", "other_launches"]
