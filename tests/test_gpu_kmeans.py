"""k-means steps of the partitioner on the GPU (lma_kmeans_assign,
lma_kmeans_update, lma_kmeans) against the k-means oracle, one step at a time
from identical inputs.  Nearest centres and squared distances are equal bit
for bit (both sides evaluate the same operations in the same order, without
fused multiply-adds).  Counts are equal; centres agree within the bound of the
summation error, because the library sums each centre's points in chunks of
4096 (then the chunks in order) while the oracle sums them in index order:
each order's sum of m values is within gamma(m-1) sum|p| of the exact sum
(gamma(m) = m u / (1 - m u), u = 2^-53), and each division adds a relative u.
At the n=524288, d=21, k=256 shape the oracle checks sampled points and
centres."""
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


U = 2.0 ** -53


def gamma(m):
    return m * U / (1.0 - m * U)


def assert_update_close(P, label, Cg, Co):
    """|Cg - Co| <= 2 gamma(m-1) sum|p| / m + 2 u |Co| per centre and
    coordinate, m = the centre's count (both sums' error bounds, both
    divisions' roundings); centres without points must be equal."""
    Cg, Co = np.asarray(Cg), np.asarray(Co)
    for c in range(Co.shape[0]):
        rows = P[label == c]
        m = rows.shape[0]
        if m == 0:
            assert np.array_equal(Cg[c], Co[c])
            continue
        bound = 2.0 * gamma(max(m - 1, 1)) * np.abs(rows).sum(axis=0) / m + 2.0 * U * np.abs(Co[c])
        assert np.all(np.abs(Cg[c] - Co[c]) <= bound), (c, np.max(np.abs(Cg[c] - Co[c]) - bound))


@pytest.mark.parametrize("name", list(CASES))
def test_assign_bit_exact_and_update_within_rounding(lib, name):
    P, C = case(name)
    print(f"case {name} n={P.shape[0]} d={P.shape[1]} k={C.shape[0]}", flush=True)
    lab, d2 = lib.kmeans_assign(P, C)
    lo, do = okm.assign(P, C)
    assert np.array_equal(np_(lab), lo) and np.array_equal(np_(d2), do)
    Cn, cnt = lib.kmeans_update(P, lo, C)
    Co, co = okm.update(P, lo, C)
    assert np.array_equal(np_(cnt), co)
    assert_update_close(P, lo, np_(Cn), Co)


@pytest.mark.parametrize("name", list(CASES))
def test_lloyd(lib, name):
    """Four Lloyd rounds: the final labels and distances are the oracle's
    assignment to the GPU's own final centres, bit for bit; the labels equal
    the oracle's Lloyd labels (no near-tie in these cases) and the centres
    agree within the rounding bound of the last update."""
    P, C = case(name)
    Cg, lg, dg = lib.kmeans(P, C, 4)
    Cg, lg, dg = np_(Cg), np_(lg), np_(dg)
    la, da = okm.assign(P, Cg)
    assert np.array_equal(lg, la) and np.array_equal(dg, da)
    Co, lo, _ = okm.lloyd(P, C, 4)
    assert np.array_equal(lg, lo)
    _, lprev, _ = okm.lloyd(P, C, 3)
    assert_update_close(P, lprev, Cg, Co)


def test_update_in_groups_of_chunks(lib, monkeypatch):
    """Partial sums held for one chunk at a time (LMA_KMEANS_PART_BYTES): the
    running sums carry the chunk order across groups, so the result is the same
    bit for bit as with every chunk's partial held at once, and within the
    rounding bound of the oracle's."""
    rng = np.random.default_rng(8)
    P = rng.uniform(0, 1, size=(13000, 3))
    C = rng.uniform(0, 1, size=(17, 3))
    lo, _ = okm.assign(P, C)
    Co, co = okm.update(P, lo, C)
    monkeypatch.setenv("LMA_KMEANS_PART_BYTES", "1")
    Cg, cg = lib.kmeans_update(P, lo, C)
    monkeypatch.delenv("LMA_KMEANS_PART_BYTES")
    Ch, ch = lib.kmeans_update(P, lo, C)
    assert np.array_equal(np_(cg), co) and np.array_equal(np_(ch), co)
    assert np.array_equal(np_(Cg), np_(Ch))
    assert_update_close(P, lo, np_(Cg), Co)


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
        sel = np.where(lg == c, 0, -1)
        Co, _ = okm.update(X, sel, Cg[c:c + 1])
        assert_update_close(X, sel, Cu[c:c + 1], Co)
