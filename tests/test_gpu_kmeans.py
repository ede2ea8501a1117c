"""k-means steps of the partitioner on the GPU (lma_kmeans_assign,
lma_kmeans_update, lma_kmeans) against the k-means oracle: labels, squared
distances, centres and counts equal bit for bit (both sides evaluate the same
operations in the same order, without fused multiply-adds).  At the n=524288,
d=21, k=256 shape the oracle checks sampled points and centres."""
import time

import numpy as np
import pytest

from oracle import kmeans as okm

pytestmark = pytest.mark.gpu

CASES = {
    "random": dict(n=5000, d=3, k=17, seed=1),
    "single_point": dict(n=1, d=1, k=1, seed=2),
    "d64_ragged": dict(n=777, d=64, k=9, seed=3),
    "more_centres_than_points": dict(n=130, d=5, k=300, seed=4),
    "duplicates_and_empty": dict(n=3000, d=2, k=40, seed=5),
}


def case(name):
    c = CASES[name]
    rng = np.random.default_rng(c["seed"])
    P = rng.uniform(0, 1, size=(c["n"], c["d"]))
    C = rng.uniform(0, 1, size=(c["k"], c["d"]))
    if name == "duplicates_and_empty":
        C[7] = C[3]            # a duplicated centre: ties go to index 3
        C[11] = 50.0           # far from every point: no points, keeps its value
        P[:5] = C[20]          # points exactly on a centre
    return P, C


def np_(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_assign_and_update_bit_exact(lib, name):
    P, C = case(name)
    print(f"case {name} n={P.shape[0]} d={P.shape[1]} k={C.shape[0]}", flush=True)
    lab, d2 = lib.kmeans_assign(P, C)
    lo, do = okm.assign(P, C)
    assert np.array_equal(np_(lab), lo) and np.array_equal(np_(d2), do)
    Cn, cnt = lib.kmeans_update(P, lo, C)
    Co, co = okm.update(P, lo, C)
    assert np.array_equal(np_(cnt), co) and np.array_equal(np_(Cn), Co)


@pytest.mark.parametrize("name", list(CASES))
def test_lloyd_bit_exact(lib, name):
    P, C = case(name)
    Cg, lg, dg = lib.kmeans(P, C, 4)
    Co, lo, do = okm.lloyd(P, C, 4)
    assert np.array_equal(np_(Cg), Co) and np.array_equal(np_(lg), lo) and np.array_equal(np_(dg), do)


def test_update_in_groups_of_chunks(lib, monkeypatch):
    """Partial sums held for one chunk at a time (LMA_KMEANS_PART_BYTES): the
    running sums carry the chunk order across groups, so the result is the same
    bit for bit."""
    rng = np.random.default_rng(8)
    P = rng.uniform(0, 1, size=(13000, 3))
    C = rng.uniform(0, 1, size=(17, 3))
    lo, _ = okm.assign(P, C)
    Co, co = okm.update(P, lo, C)
    monkeypatch.setenv("LMA_KMEANS_PART_BYTES", "1")
    Cg, cg = lib.kmeans_update(P, lo, C)
    monkeypatch.delenv("LMA_KMEANS_PART_BYTES")
    assert np.array_equal(np_(cg), co) and np.array_equal(np_(Cg), Co)


def test_workload_shape_sampled(lib):
    """n=524288 points in 21-D from a mixture of 32 Gaussians, k=256 centres
    started at random rows, 10 Lloyd rounds on the GPU.  The oracle then checks
    4096 sampled points (nearest centre and distance against the final
    centres) and 16 sampled centres (the update from the final labels)."""
    import torch
    rng = np.random.default_rng(14114510)
    cen = rng.uniform(0, 1, size=(32, 21))
    X = cen[rng.integers(32, size=524288)] + 0.2 * rng.standard_normal((524288, 21))
    C0 = X[np.sort(rng.choice(524288, 256, replace=False))]
    Xd = torch.as_tensor(X, device="cuda")
    lib.kmeans(Xd, C0, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Cg, lg, dg = lib.kmeans(Xd, C0, 10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"  10 Lloyd rounds + final assignment, n=524288 d=21 k=256: {dt * 1e3:.1f} ms", flush=True)
    Cg, lg, dg = np_(Cg), np_(lg), np_(dg)
    idx = np.sort(rng.choice(524288, 4096, replace=False))
    lo, do = okm.assign(X[idx], Cg)
    assert np.array_equal(lg[idx], lo) and np.array_equal(dg[idx], do)
    Cu, cnt = lib.kmeans_update(Xd, lg, Cg)
    Cu, cnt = np_(Cu), np_(cnt)
    assert np.array_equal(cnt, np.bincount(lg, minlength=256))
    for c in rng.choice(256, 16, replace=False):
        Co, _ = okm.update(X, np.where(lg == c, 0, -1), Cg[c:c + 1])
        assert np.array_equal(Cu[c], Co[0])
