"""Pins for the partition oracle (oracle/partition.py): hand-worked cases of
the bounded assignment, its reduction to the plain nearest-centre assignment
when the bounds do not bind, the bounds themselves, the properties each phase
guarantees (every strictly nearer centre of a point is full after the upper
phase; the points moved to a short centre are nearer to it than every point
left with a centre that could still give), the exact integer draw of the
seeding (closed-form pick counts, the first index, no point drawn twice, the
quantised weights' range), and the composed partition (a permutation,
block-contiguous, stable, bounded, chain-ordered, test points at their
nearest block centre)."""
import numpy as np
import pytest

from oracle import kmeans as okm
from oracle import partition as opart


def line(points):
    return np.asarray(points, dtype=np.float64)[:, None]


# --- bounded assignment ------------------------------------------------------

def test_upper_phase_by_hand():
    """Points 0, 1, 2, 10 and centres 0.5, 9 with at most 2 points per centre.
    Round 1: points 0, 1, 2 propose to centre 0 (distances 0.25, 0.25, 2.25),
    point 10 to centre 1; centre 0 keeps its 2 nearest (0 and 1, tied at 0.25:
    lower index first) and closes.  Round 2: point 2 proposes to centre 1."""
    lab, rounds = opart.bounded_assign(line([0, 1, 2, 10]), line([0.5, 9]), 0, 2)
    assert lab.tolist() == [0, 0, 1, 1] and rounds == 2


def test_tie_at_the_cut_goes_to_the_lower_index():
    """Centre 0 (at 0) with room for two gets three proposers: the point at 0.2
    and two points at distance exactly 1 (at 1 and -1).  It keeps 0.2 and, of
    the tied two, the one with the lower index, whichever side it lies on."""
    lab, _ = opart.bounded_assign(line([1, -1, 0.2, 50]), line([0, 40]), 0, 2)
    assert lab.tolist() == [0, 1, 0, 1]
    lab, _ = opart.bounded_assign(line([-1, 1, 0.2, 50]), line([0, 40]), 0, 2)
    assert lab.tolist() == [0, 1, 0, 1]


def test_lower_phase_by_hand():
    """Points 0, 1, 2, 3, 10, centres 1 and 10, sizes in [2, 4]: the upper phase
    gives centre 0 the first four points and centre 1 only point 10; centre 1
    then takes the nearest point of centre 0 (point 3, distance 49)."""
    lab, _ = opart.bounded_assign(line([0, 1, 2, 3, 10]), line([1, 10]), 2, 4)
    assert lab.tolist() == [0, 0, 0, 1, 1]


def test_lower_phase_stops_taking_from_a_donor_at_lo():
    """Points 0..4 and 50, 51, 52, centres 2, 51, 100, sizes in [lo, 5].
    The upper phase gives centre 0 the points 0..4, centre 1 the points
    50..52 and centre 2 nothing.
    lo = 2: centre 2 needs two points.  The nearest, 52, comes from centre 1,
    which then holds 2 = lo and gives no more, so the next one is 4 (from
    centre 0) although 51 is nearer.
    lo = 3 (with 100 added as a ninth point): centre 2 holds 100 and needs two
    more; centre 1 holds 3 = lo and gives nothing, centre 0 gives 4 and 3."""
    P = line([0, 1, 2, 3, 4, 50, 51, 52])
    C = line([2, 51, 100])
    lab, _ = opart.bounded_assign(P, C, 2, 5)
    assert lab.tolist() == [0, 0, 0, 0, 2, 1, 1, 2]
    lab, _ = opart.bounded_assign(line([0, 1, 2, 3, 4, 50, 51, 52, 100]), C, 3, 5)
    assert lab.tolist() == [0, 0, 0, 2, 2, 1, 1, 1, 2]


@pytest.mark.parametrize("seed,n,d,k", [(1, 500, 2, 7), (2, 800, 3, 16), (3, 300, 5, 4)])
def test_loose_bounds_are_the_nearest_centre(seed, n, d, k):
    rng = np.random.default_rng(seed)
    P, C = rng.uniform(size=(n, d)), rng.uniform(size=(k, d))
    lab, rounds = opart.bounded_assign(P, C, 0, n)
    assert np.array_equal(lab, okm.assign(P, C)[0]) and rounds == 1


@pytest.mark.parametrize("seed,n,k,lo,hi", [(4, 600, 8, 60, 90), (5, 1000, 10, 100, 100), (6, 700, 7, 0, 101),
                                             (7, 900, 12, 70, 80)])
def test_bounds_and_phase_properties(seed, n, k, lo, hi):
    rng = np.random.default_rng(seed)
    # clustered points so that both bounds bind
    cen = rng.uniform(size=(3, 2))
    P = cen[rng.integers(3, size=n)] + 0.05 * rng.standard_normal((n, 2))
    C = P[rng.choice(n, k, replace=False)]
    lab, _ = opart.bounded_assign(P, C, lo, hi)
    cnt = np.bincount(lab, minlength=k)
    assert cnt.min() >= lo and cnt.max() <= hi and cnt.sum() == n
    D = np.stack([okm.sqdist_to(P, C[c]) for c in range(k)], axis=1)
    # upper phase alone (lo = 0): every centre strictly nearer than a point's
    # own is full
    up, _ = opart.bounded_assign(P, C, 0, hi)
    ucnt = np.bincount(up, minlength=k)
    for i in range(n):
        nearer = D[i] < D[i, up[i]]
        assert np.all(ucnt[nearer] == hi)


def test_points_moved_to_a_short_centre_are_its_nearest_available():
    rng = np.random.default_rng(8)
    P = np.vstack([rng.normal(0, 0.1, size=(300, 2)), rng.normal(3, 0.1, size=(10, 2))])
    C = np.array([[0.0, 0.0], [0.1, 0.0], [3.0, 3.0]])
    lo, hi = 60, 200
    up, _ = opart.bounded_assign(P, C, 0, hi)
    lab, _ = opart.bounded_assign(P, C, lo, hi)
    moved = np.flatnonzero((lab == 2) & (up != 2))
    assert moved.size == lo - np.sum(up == 2)
    cnt = np.bincount(lab, minlength=3)
    d2 = okm.sqdist_to(P, C[2])
    # every point left with a centre that still holds more than lo is no
    # nearer to centre 2 than the farthest moved point
    rest = np.flatnonzero((lab != 2) & (cnt[lab] > lo))
    assert d2[rest].min() >= d2[moved].max()


# --- seeding ------------------------------------------------------------------

def test_pick_counts_equal_the_weights():
    """Weights 1, 3, 4 (total 8): the 8 draws r = j 2^29, j = 0..7, give the
    targets 0..7 exactly, so point i is drawn w_i times."""
    w = np.array([1, 3, 4], dtype=np.uint64)
    picks = [opart.pick(w, j << 29, 3) for j in range(8)]
    assert np.bincount(picks, minlength=3).tolist() == [1, 3, 4]
    assert opart.pick(np.zeros(3, dtype=np.uint64), 3 << 30, 3) == 2      # all zero: floor(r n / 2^32)


def test_quantised_weights():
    n = 1000
    rng = np.random.default_rng(9)
    dmin = rng.uniform(0, 7.3, size=n)
    dmin[5] = 0.0
    w = opart.quantise(dmin, n)
    W = opart.weight_bits(n)
    assert W == 63 - 10
    top = int(w[np.argmax(dmin)])
    assert 2 ** (W - 1) <= top < 2 ** W and w[5] == 0
    assert sum(int(v) for v in w) < 2 ** 63
    # proportional to the distances within the truncation
    assert np.all(np.abs(w.astype(np.float64) / top - dmin / dmin.max()) <= 2.0 ** (2 - W))


def test_seeding_draws_distinct_points_and_starts_where_told():
    rng = np.random.default_rng(10)
    P = rng.uniform(size=(400, 3))
    rand = rng.integers(0, 2 ** 32, size=50, dtype=np.uint64)
    C, idx = opart.seed(P, 50, rand)
    assert idx[0] == (int(rand[0]) * 400) >> 32
    assert len(set(idx.tolist())) == 50 and np.array_equal(C, P[idx])


def test_seeding_reaches_separated_clusters():
    """Four tight clusters far apart: D^2 sampling puts one of the first four
    centres in each cluster for any draw whose weights are not vanishingly
    small (here, twenty draws)."""
    rng = np.random.default_rng(11)
    cen = np.array([[0, 0], [100, 0], [0, 100], [100, 100]], dtype=np.float64)
    lab = rng.integers(4, size=2000)
    P = cen[lab] + 0.01 * rng.standard_normal((2000, 2))
    for t in range(20):
        rand = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)
        _, idx = opart.seed(P, 4, rand)
        assert sorted(lab[idx].tolist()) == [0, 1, 2, 3]


# --- composed partition --------------------------------------------------------

def test_partition_properties():
    rng = np.random.default_rng(12)
    cen = rng.uniform(size=(5, 3))
    X = cen[rng.integers(5, size=3000)] + 0.1 * rng.standard_normal((3000, 3))
    U = cen[rng.integers(5, size=400)] + 0.1 * rng.standard_normal((400, 3))
    M, lo, hi = 12, 150, 400
    rand = rng.integers(0, 2 ** 32, size=M, dtype=np.uint64)
    r = opart.partition(X, M, lo, hi, 5, rand, U=U)
    perm, bp = r["perm"], r["block_ptr"]
    assert sorted(perm.tolist()) == list(range(3000))
    sizes = np.diff(bp)
    assert bp[0] == 0 and bp[-1] == 3000 and sizes.min() >= lo and sizes.max() <= hi
    rank = np.empty(M, dtype=np.int64)
    rank[r["chain"]] = np.arange(M)
    blk = rank[r["label"]]
    for m in range(M):
        seg = perm[bp[m]:bp[m + 1]]
        assert np.all(blk[seg] == m) and np.all(np.diff(seg) > 0)        # stable
    # block centres are the block means, in chain order
    for m in range(M):
        assert np.allclose(r["C_blocks"][m], X[perm[bp[m]:bp[m + 1]]].mean(axis=0), rtol=1e-12, atol=1e-14)
    # test points: nearest block centre (away from near-ties), block-contiguous
    up, ubp = r["u_perm"], r["u_block_ptr"]
    D = np.linalg.norm(U[:, None, :] - r["C_blocks"][None], axis=2)
    srt = np.sort(D, axis=1)
    clear = srt[:, 1] - srt[:, 0] > 1e-9
    ublk = np.empty(400, dtype=np.int64)
    for m in range(M):
        ublk[up[ubp[m]:ubp[m + 1]]] = m
    assert np.array_equal(ublk[clear], np.argmin(D, axis=1)[clear])
    assert sorted(up.tolist()) == list(range(400))
