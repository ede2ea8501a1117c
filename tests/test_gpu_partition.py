"""Block partition on the GPU (lma_kmeans_seed, lma_bounded_assign,
lma_partition) against the partition oracle, one step at a time from identical
inputs: seeding indices, bounded labels, proposal rounds, chain order, the
permutations and block pointers are equal bit for bit (every decision is taken
on exact quantities on both sides); centres from a centre update agree within
the bound of the summation error (the library sums in chunks).  The composed
call equals the composition of its steps, and the whole oracle partition from
the same random integers.  At the n=524288, d=21, M=256 shape the oracle checks
properties and sampled points, and the partition is timed."""
import time

import numpy as np
import pytest

from oracle import kmeans as okm
from oracle import partition as opart

pytestmark = pytest.mark.gpu


def np_(t):
    return t.cpu().numpy()


def line(points):
    return np.asarray(points, dtype=np.float64)[:, None]


def clustered(seed, n, d, nc=6, spread=0.1):
    rng = np.random.default_rng(seed)
    cen = rng.uniform(size=(nc, d))
    return cen[rng.integers(nc, size=n)] + spread * rng.standard_normal((n, d)), rng


SEED_CASES = {
    "one_point": (1, 1, 1),
    "k_equals_n": (50, 3, 50),
    "uniform": (5000, 4, 64),
    "d64": (700, 64, 20),
    "several_blocks_of_threads": (100000, 8, 200),
}


@pytest.mark.parametrize("name", list(SEED_CASES))
def test_seeding_equals_the_oracle(lib, name):
    n, d, k = SEED_CASES[name]
    print(f"case seed {name} n={n} d={d} k={k}", flush=True)
    rng = np.random.default_rng(n + d + k)
    P = rng.uniform(size=(n, d))
    rand = rng.integers(0, 2 ** 32, size=k, dtype=np.uint64).astype(np.uint32)
    C, idx = lib.kmeans_seed(P, k, rand)
    Co, io = opart.seed(P, k, rand)
    assert np.array_equal(np_(idx), io) and np.array_equal(np_(C), Co)


def test_seeding_when_every_point_is_a_centre(lib):
    """All points equal: every weight is 0 after the first draw, so each draw
    falls back to floor(r n / 2^32)."""
    P = np.ones((10, 2))
    rand = np.array([5, 2 ** 31, 3 * 2 ** 30], dtype=np.uint32)
    _, idx = lib.kmeans_seed(P, 3, rand)
    _, io = opart.seed(P, 3, rand)
    assert np.array_equal(np_(idx), io) and np_(idx).tolist() == [0, 5, 7]


HAND = [
    (line([0, 1, 2, 10]), line([0.5, 9]), 0, 2, [0, 0, 1, 1]),
    (line([1, -1, 0.2, 50]), line([0, 40]), 0, 2, [0, 1, 0, 1]),
    (line([-1, 1, 0.2, 50]), line([0, 40]), 0, 2, [0, 1, 0, 1]),
    (line([0, 1, 2, 3, 10]), line([1, 10]), 2, 4, [0, 0, 0, 1, 1]),
    (line([0, 1, 2, 3, 4, 50, 51, 52]), line([2, 51, 100]), 2, 5, [0, 0, 0, 0, 2, 1, 1, 2]),
    (line([0, 1, 2, 3, 4, 50, 51, 52, 100]), line([2, 51, 100]), 3, 5, [0, 0, 0, 2, 2, 1, 1, 1, 2]),
]


@pytest.mark.parametrize("i", range(len(HAND)))
def test_bounded_assignment_hand_cases(lib, i):
    P, C, lo, hi, want = HAND[i]
    lab, cnt, _ = lib.bounded_assign(P, C, lo, hi)
    assert np_(lab).tolist() == want
    assert np_(cnt).tolist() == np.bincount(want, minlength=C.shape[0]).tolist()


BOUNDED = {
    "loose": (3000, 3, 12, 0, 3000),
    "upper_binds": (6000, 2, 16, 0, 420),
    "both_bind": (8000, 5, 20, 300, 520),
    "equal_sizes": (4096, 4, 16, 256, 256),
    "many_centres": (30000, 3, 300, 60, 150),
}


@pytest.mark.parametrize("name", list(BOUNDED))
def test_bounded_assignment_equals_the_oracle(lib, name):
    n, d, k, lo, hi = BOUNDED[name]
    print(f"case bounded {name} n={n} d={d} k={k} lo={lo} hi={hi}", flush=True)
    P, rng = clustered(len(name), n, d)
    C = P[rng.choice(n, k, replace=False)]
    lab, cnt, rounds = lib.bounded_assign(P, C, lo, hi)
    lo_, ro = opart.bounded_assign(P, C, lo, hi)
    print(f"  rounds {rounds}", flush=True)
    assert np.array_equal(np_(lab), lo_) and rounds == ro
    c = np_(cnt)
    assert np.array_equal(c, np.bincount(lo_, minlength=k)) and c.min() >= lo and c.max() <= hi


def test_bounded_assignment_rejects_impossible_bounds(lib):
    P = np.zeros((10, 2))
    C = np.zeros((3, 2))
    for lo, hi in ((4, 5), (0, 3), (3, 2)):
        with pytest.raises(lib.LmaError) as e:
            lib.bounded_assign(P, C, lo, hi)
        assert e.value.status == lib.LMA_E_ARG
    P[3, 1] = np.nan
    with pytest.raises(lib.LmaError) as e:
        lib.bounded_assign(P, C, 0, 5)
    assert e.value.status == lib.LMA_E_ARG


def steps_on_gpu(lib, X, M, lo, hi, iters, rand):
    """The partition's steps through their own entry points."""
    C0, idx = lib.kmeans_seed(X, M, rand)
    C, _, _ = lib.kmeans(X, C0, iters)
    label, cnt, rounds = lib.bounded_assign(X, C, lo, hi)
    Cb, _ = lib.kmeans_update(X, label, C)
    return np_(idx), np_(C), np_(label), np_(Cb)


def test_partition_equals_its_steps_and_the_oracle(lib):
    X, rng = clustered(3, 20000, 5)
    U = X[rng.choice(20000, 3000, replace=False)] + 0.01 * rng.standard_normal((3000, 5))
    M, lo, hi, iters = 16, 900, 1600, 5
    rand = rng.integers(0, 2 ** 32, size=M, dtype=np.uint64).astype(np.uint32)
    print(f"case partition n=20000 d=5 M={M} lo={lo} hi={hi}", flush=True)
    r = lib.partition(X, M, lo, hi, iters, rand, U=U)
    perm, bp, uperm, ubp, cen = np_(r["perm"]), r["block_ptr"], np_(r["u_perm"]), r["u_block_ptr"], np_(r["centres"])
    # the steps, on the GPU and in the oracle from the GPU's inputs to each step
    idx, C, label, Cb = steps_on_gpu(lib, X, M, lo, hi, iters, rand)
    assert np.array_equal(idx, opart.seed(X, M, rand)[1])
    assert np.array_equal(label, opart.bounded_assign(X, C, lo, hi)[0])
    chain = okm.chain_order(Cb)
    assert np.array_equal(chain, lib.chain_order(Cb))
    rank = np.empty(M, dtype=np.int64)
    rank[chain] = np.arange(M)
    assert np.array_equal(cen, Cb[chain])
    assert np.array_equal(perm, np.argsort(rank[label], kind="stable"))
    assert np.array_equal(bp, np.r_[0, np.cumsum(np.bincount(rank[label], minlength=M))])
    ulab = okm.assign(U, Cb)[0]
    assert np.array_equal(uperm, np.argsort(rank[ulab], kind="stable"))
    assert np.array_equal(ubp, np.r_[0, np.cumsum(np.bincount(rank[ulab], minlength=M))])
    # the whole oracle partition from the same random integers
    o = opart.partition(X, M, lo, hi, iters, rand, U=U)
    assert np.array_equal(perm, o["perm"]) and np.array_equal(bp, o["block_ptr"])
    assert np.array_equal(uperm, o["u_perm"]) and np.array_equal(ubp, o["u_block_ptr"])
    assert np.max(np.abs(cen - o["C_blocks"])) <= 1e-12 * np.max(np.abs(o["C_blocks"]))


def test_partition_without_test_points_and_with_one_block(lib):
    X, rng = clustered(4, 3000, 3)
    rand = rng.integers(0, 2 ** 32, size=1, dtype=np.uint64).astype(np.uint32)
    r = lib.partition(X, 1, 0, 3000, 3, rand)
    assert np.array_equal(np_(r["perm"]), np.arange(3000))
    assert r["block_ptr"].tolist() == [0, 3000] and r["u_block_ptr"].tolist() == [0, 0]


def test_workload_shape(lib):
    """n=524288 points in 21-D (mixture of 32 Gaussians), M=256 blocks of
    1024..3072 points, 10 Lloyd rounds, 65536 test points: timed; the oracle
    checks the block sizes, the permutations, the stable order, the steps'
    composition, sampled test points and sampled block centres."""
    import torch
    rng = np.random.default_rng(14114510)
    cen = rng.uniform(0, 1, size=(32, 21))
    X = cen[rng.integers(32, size=524288)] + 0.2 * rng.standard_normal((524288, 21))
    U = cen[rng.integers(32, size=65536)] + 0.2 * rng.standard_normal((65536, 21))
    M, lo, hi, iters = 256, 1024, 3072, 10
    rand = rng.integers(0, 2 ** 32, size=M, dtype=np.uint64).astype(np.uint32)
    Xd, Ud = torch.as_tensor(X, device="cuda"), torch.as_tensor(U, device="cuda")
    lib.partition(Xd, M, lo, hi, iters, rand, U=Ud)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = lib.partition(Xd, M, lo, hi, iters, rand, U=Ud)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    perm, bp, uperm, ubp, cenb = np_(r["perm"]), r["block_ptr"], np_(r["u_perm"]), r["u_block_ptr"], np_(r["centres"])
    sizes = np.diff(bp)
    print(f"  partition n=524288 d=21 M=256 (+65536 test points): {dt * 1e3:.1f} ms; block sizes "
          f"{sizes.min()}..{sizes.max()}", flush=True)
    assert sizes.min() >= lo and sizes.max() <= hi and bp[-1] == 524288
    assert np.array_equal(np.sort(perm), np.arange(524288)) and np.array_equal(np.sort(uperm), np.arange(65536))
    # composition of the steps, bit for bit
    idx, C, label, Cb = steps_on_gpu(lib, Xd, M, lo, hi, iters, rand)
    chain = lib.chain_order(Cb)
    assert np.array_equal(chain, okm.chain_order(Cb))
    rank = np.empty(M, dtype=np.int64)
    rank[chain] = np.arange(M)
    assert np.array_equal(cenb, Cb[chain])
    assert np.array_equal(perm, np.argsort(rank[label], kind="stable"))
    # sampled test points: nearest block centre
    s = np.sort(rng.choice(65536, 2048, replace=False))
    ublk = np.empty(65536, dtype=np.int64)
    for m in range(M):
        ublk[uperm[ubp[m]:ubp[m + 1]]] = m
    assert np.array_equal(ublk[s], rank[okm.assign(U[s], Cb)[0]])
    # sampled block centres: the mean of their block within rounding
    for m in rng.choice(M, 8, replace=False):
        pts = X[perm[bp[m]:bp[m + 1]]]
        Co, _ = okm.update(pts, np.zeros(pts.shape[0], dtype=np.int64), cenb[m:m + 1])
        assert np.max(np.abs(cenb[m] - Co[0])) <= 1e-13 * max(1.0, np.max(np.abs(Co[0])))
