"""The C-ABI library builds, loads and exports every symbol that include/lma.h
declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import numpy as np
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
    assert set(header_functions("lma_part.h")) == set(lma.PART_EXPORTS)


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(lma.LIB_PATH):
        pytest.fail("liblma.so not built (run paper_1411_4510_amd.build)")
    return ctypes.CDLL(lma.LIB_PATH)


def test_library_exports_every_declared_symbol(so):
    for name in header_functions() + header_functions("lma_ds.h") + header_functions("lma_part.h"):
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


def test_failed_block_is_reset_by_every_entry_point(so):
    """lma_failed_block names no block (-3) after a call that did not fail on a
    factor: each entry point resets it when it starts."""
    so.lma_failed_block.restype = ctypes.c_int64
    so.lma_fit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    so.lma_fit.restype = ctypes.c_int
    so.lma_predict.restype = ctypes.c_int
    so.lma_predict.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    so.lma_lml.restype = ctypes.c_int
    so.lma_lml.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert so.lma_failed_block() == -3
    h = ctypes.c_void_p()
    assert so.lma_fit(None, None, ctypes.byref(h)) == lma.LMA_E_ARG
    assert so.lma_failed_block() == -3
    assert so.lma_predict(None, 1, None, None, None, None, None) == lma.LMA_E_ARG
    assert so.lma_failed_block() == -3
    v = ctypes.c_double()
    assert so.lma_lml(None, ctypes.byref(v), None, None) == lma.LMA_E_ARG
    assert so.lma_failed_block() == -3


BAD_PROBLEMS = [
    ("d = 0", dict(d=0)),
    ("d = 65", dict(d=65)),
    ("n = 0", dict(n=0)),
    ("s = 0", dict(s=0)),
    ("B < 0", dict(B=-1)),
    ("more blocks than points", dict(M=20)),
    ("block_ptr not ending at n", dict(bp=[0, 3, 6, 9])),
    ("empty block", dict(bp=[0, 3, 3, 10])),
    ("unknown precision", dict(precision=7)),
    ("reserved field set", dict(reserved=1)),
    ("non-finite hyperparameter", dict(log_hyp=[0.0, float("nan"), 0.0, 0.0])),
    ("non-finite prior mean", dict(prior_mean=float("inf"))),
    ("support set beyond 8192", dict(s=8193)),
    ("NULL X", dict(X=None)),
]


@pytest.mark.parametrize("what,kw", BAD_PROBLEMS, ids=[b[0] for b in BAD_PROBLEMS])
def test_bad_problems_rejected_on_the_host(so, what, kw):
    """Argument errors come back as LMA_E_ARG with a message before any device
    call (the arrays are host dummies: only their presence is checked)."""
    so.lma_fit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    so.lma_fit.restype = ctypes.c_int
    so.lma_last_error.restype = ctypes.c_char_p
    dummy = (ctypes.c_double * 64)()
    bp = (ctypes.c_int64 * 4)(*kw.get("bp", [0, 3, 6, 10]))
    lh = (ctypes.c_double * 4)(*kw.get("log_hyp", [0.0, 0.0, 0.0, -2.0]))
    pr = lma._Problem()
    pr.n, pr.d, pr.s = kw.get("n", 10), kw.get("d", 2), kw.get("s", 4)
    pr.M, pr.B = kw.get("M", 3), kw.get("B", 1)
    addr = ctypes.cast(dummy, ctypes.c_void_p).value
    pr.X = kw.get("X", addr)
    pr.y = addr
    pr.S = addr
    pr.block_ptr = ctypes.cast(bp, ctypes.POINTER(ctypes.c_int64))
    pr.log_hyp = ctypes.cast(lh, ctypes.POINTER(ctypes.c_double))
    pr.prior_mean = kw.get("prior_mean", 0.0)
    pr.precision = kw.get("precision", 0)
    pr.reserved = kw.get("reserved", 0)
    h = ctypes.c_void_p()
    assert so.lma_fit(ctypes.byref(pr), None, ctypes.byref(h)) == lma.LMA_E_ARG, what
    assert not h.value
    assert so.lma_last_error().decode()


def test_binding_struct_matches_header_layout():
    # lma_problem: 5 int64, 6 pointers/doubles in order, then int32 x2 and int64
    assert ctypes.sizeof(lma._Problem) == 5 * 8 + 5 * 8 + 8 + 4 + 4 + 8


def test_profile_struct_matches_header_layout():
    # lma_profile: 6 doubles, 2 int64, 4 doubles, 2 int64
    assert ctypes.sizeof(lma.Profile) == 14 * 8
    names = [f for f, _ in lma.Profile._fields_]
    assert names[:8] == ["update_ms", "diag_ms", "trsm_ms", "other_ms", "update_alg_flops",
                         "update_alg_flops_f64", "update_launches", "other_launches"]


KMEANS_BAD = [
    ("d = 0", dict(d=0)),
    ("d = 65", dict(d=65)),
    ("k = 0", dict(k=0)),
    ("k beyond 65536", dict(k=65537)),
    ("n < 0", dict(n=-1)),
    ("NULL points", dict(P=None)),
    ("NULL centres", dict(C=None)),
    ("NULL labels", dict(label=None)),
    ("iters < 0", dict(iters=-1)),
]


@pytest.mark.parametrize("what,kw", KMEANS_BAD, ids=[w for w, _ in KMEANS_BAD])
def test_kmeans_argument_errors_without_gpu(so, what, kw):
    """The k-means entry points reject bad shapes and NULL arrays on the host
    (no device call is made for them)."""
    vp = ctypes.c_void_p
    so.lma_kmeans.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    so.lma_kmeans.restype = ctypes.c_int
    so.lma_last_error.restype = ctypes.c_char_p
    dummy = vp(0x1000)  # never dereferenced: every case fails its host check first
    a = dict(P=dummy, n=10, d=2, C=dummy, k=3, iters=1, label=dummy)
    a.update(kw)
    st = so.lma_kmeans(a["P"], a["n"], a["d"], a["C"], a["k"], a["iters"], a["label"], None, None)
    assert st == lma.LMA_E_ARG, what
    assert so.lma_last_error().decode()


@pytest.mark.parametrize("k,d,seed", [(256, 21, 1), (1, 3, 2), (2, 1, 3), (97, 64, 4)])
def test_chain_order_matches_oracle_bit_for_bit(k, d, seed):
    """lma_chain_order is a host function (no device work): the same order as
    the oracle, including duplicated centres (ties to the lowest index)."""
    from oracle import kmeans as okm
    rng = np.random.default_rng(seed)
    C = rng.uniform(0, 1, size=(k, d))
    if k > 4:
        C[3] = C[1]
    assert np.array_equal(lma.chain_order(C), okm.chain_order(C))


def test_chain_order_argument_errors(so):
    so.lma_chain_order.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    so.lma_chain_order.restype = ctypes.c_int
    buf = (ctypes.c_double * 8)()
    out = (ctypes.c_int32 * 4)()
    assert so.lma_chain_order(buf, 0, 2, out) == lma.LMA_E_ARG
    assert so.lma_chain_order(buf, 4, 0, out) == lma.LMA_E_ARG
    assert so.lma_chain_order(None, 4, 2, out) == lma.LMA_E_ARG
    assert so.lma_chain_order(buf, 4, 2, None) == lma.LMA_E_ARG
