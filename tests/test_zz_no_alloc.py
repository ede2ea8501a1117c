"""The allocation-free centre update (lma_kmeans_update_noalloc), called
through the C ABI, against lma_kmeans_update on the same inputs: the same
centres and counts bit for bit (the same kernels; running sums carry the chunk
order across groups of chunks, so the group size the fixed scratch allows does
not change the result), on two calls in a row, the second with a smaller
input; sizes beyond the scratch are rejected."""
import ctypes

import numpy as np
import pytest

from oracle import kmeans as okm

pytestmark = pytest.mark.gpu


def call_noalloc(lib, torch, P, lab, C):
    so = lib.load()
    Pd = torch.as_tensor(P, device="cuda")
    ld = torch.as_tensor(lab, device="cuda").to(torch.int32).contiguous()
    Cd = torch.as_tensor(C, device="cuda").clone()
    cnt = torch.empty(C.shape[0], dtype=torch.int64, device="cuda")
    st = so.lma_kmeans_update_noalloc(ctypes.c_void_p(Pd.data_ptr()), P.shape[0], P.shape[1],
                                      ctypes.c_void_p(ld.data_ptr()), C.shape[0], ctypes.c_void_p(Cd.data_ptr()),
                                      ctypes.c_void_p(cnt.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, Cd.cpu().numpy(), cnt.cpu().numpy()


def test_noalloc_update_matches_the_allocating_one(lib):
    import torch
    # first call: k*d = 65536 (two groups of chunks in the 16 MiB scratch)
    # second call: a smaller input on the same scratch
    for n, d, k, seed in ((200000, 32, 2048, 1), (10000, 5, 300, 2)):
        print(f"case noalloc n={n} d={d} k={k}", flush=True)
        rng = np.random.default_rng(seed)
        P = rng.standard_normal((n, d))
        lab = rng.integers(-1, k, size=n).astype(np.int32)   # -1: a point of no centre
        C = rng.standard_normal((k, d))
        st, Cn, cn = call_noalloc(lib, torch, P, lab, C)
        assert st == lib.LMA_OK, lib.load().lma_last_error()
        Ca, ca = lib.kmeans_update(P, lab, C)
        assert np.array_equal(cn, ca.cpu().numpy()) and np.array_equal(Cn, Ca.cpu().numpy())
        Co, co = okm.update(P, lab, C)
        assert np.array_equal(cn, co)
        assert np.max(np.abs(Cn - Co)) <= 1e-12 * max(1.0, np.max(np.abs(Co)))


def test_noalloc_update_rejects_sizes_beyond_the_scratch(lib):
    import torch
    P = np.zeros((10, 64))
    st, _, _ = call_noalloc(lib, torch, P, np.zeros(10, np.int32), np.zeros((20000, 64)))
    assert st == lib.LMA_E_ARG
    assert b"allocation-free" in lib.load().lma_last_error()
