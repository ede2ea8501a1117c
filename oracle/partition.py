"""Block partition of the inputs, written out plainly (oracle; test
infrastructure only).

LMA needs the training inputs D and the test inputs U partitioned into M
blocks, with the blocks ordered so that the next B blocks of each are its most
correlated neighbours (section "Low-Rank-cum-Markov Approximation": the paper
takes the clustering of D and U from earlier work without specifying it, and
D^B_m is the set of the B blocks after D_m).  The partition computed here:

  1. seeding (k-means++, D^2 sampling): the first centre is point
     floor(r_0 n / 2^32); each further centre j is drawn with probability
     proportional to every point's squared distance to its nearest centre so
     far.  The weights are those squared distances quantised to integers: with
     e the binary exponent of their maximum (max = f 2^e, 0.5 <= f < 1) and
     W = 63 - bitlength(n), weight_i = floor(dmin_i 2^(W - e)), so the total
     stays below 2^63 and is exact whatever the summation order.  With T the
     total, target = floor(r_j T / 2^32) and the centre is the first point
     whose running weight sum exceeds the target.  r_0 .. r_{k-1} are the
     caller's random 32-bit integers.  (If every weight is 0, i.e. every point
     sits on a chosen centre, the pick is floor(r_j n / 2^32).)
  2. Lloyd's iteration from those centres (kmeans.lloyd).
  3. capacity-bounded assignment: every block ends with lo..hi points.
     Upper bound, in rounds: every point not yet placed proposes to its
     nearest centre among those holding fewer than hi points; a centre with
     room for r more points accepts all its proposers if they are at most r,
     else the r nearest (smallest squared distance, ties to the lower point
     index).  Rounds repeat until every point is placed.
     Lower bound, centre by centre in increasing index: while centre c holds
     fewer than lo points, the point nearest to c (ties to the lower index)
     among the points of other centres that hold more than lo points moves to
     c.
  4. block centres: the mean of each block's points (kmeans.update).
  5. block order: the nearest-neighbour chain through the block centres
     (kmeans.chain_order); block m of the partition is the chain's m-th centre.
  6. test points: each goes to the block of its nearest block centre
     (unbounded).
  7. the permutation: training points sorted by block, stably (points of one
     block keep their index order); the same for the test points.

Squared distances and nearest centres follow kmeans.sqdist_to / kmeans.assign
(coordinates summed in increasing order, ties to the lower centre index).
"""
import numpy as np

from . import kmeans as okm


def weight_bits(n):
    """W = 63 - bitlength(n): n weights below 2^W sum to less than 2^63."""
    return 63 - int(n).bit_length()


def quantise(dmin, n):
    """Integer sampling weights floor(dmin 2^(W - e)), e the binary exponent of
    max(dmin); all zero when the maximum is 0."""
    mx = float(np.max(dmin))
    if not mx > 0.0:
        return np.zeros(dmin.shape[0], dtype=np.uint64)
    _, e = np.frexp(mx)
    scaled = np.ldexp(dmin, weight_bits(n) - int(e))      # exact: a power of two
    return np.floor(scaled).astype(np.uint64)


def pick(weights, r, n):
    """The first index whose running weight sum exceeds floor(r T / 2^32)."""
    total = 0
    for w in weights.tolist():
        total += w
    if total == 0:
        return (int(r) * n) >> 32
    target = (int(r) * total) >> 32                       # exact integer product
    run = 0
    for i, w in enumerate(weights.tolist()):
        run += w
        if run > target:
            return i
    raise AssertionError("target beyond the total")


def seed(P, k, rand):
    """k-means++ centres (rows of P) and their point indices."""
    P = np.asarray(P, dtype=np.float64)
    n = P.shape[0]
    rand = np.asarray(rand, dtype=np.uint64)
    idx = [(int(rand[0]) * n) >> 32]
    dmin = okm.sqdist_to(P, P[idx[0]])
    for j in range(1, k):
        i = pick(quantise(dmin, n), int(rand[j]), n)
        idx.append(i)
        dmin = np.minimum(dmin, okm.sqdist_to(P, P[i]))
    idx = np.asarray(idx, dtype=np.int64)
    return P[idx].copy(), idx


def nearest_open(P, C, open_):
    """Nearest centre among the open ones (ties to the lower index) and its
    squared distance; a point with no finite distance takes the lowest open
    centre at distance +inf."""
    best = np.full(P.shape[0], np.inf)
    arg = np.full(P.shape[0], int(np.flatnonzero(open_)[0]), dtype=np.int64)
    for c in np.flatnonzero(open_):
        acc = okm.sqdist_to(P, C[c])
        better = acc < best
        best[better] = acc[better]
        arg[better] = c
    return arg, best


def bounded_assign(P, C, lo, hi):
    """Labels with lo <= block size <= hi, and the number of proposal rounds."""
    P, C = np.asarray(P, dtype=np.float64), np.asarray(C, dtype=np.float64)
    n, k = P.shape[0], C.shape[0]
    assert 0 <= lo <= hi and hi >= 1 and k * lo <= n <= k * hi
    label = np.full(n, -1, dtype=np.int64)
    count = np.zeros(k, dtype=np.int64)
    rounds = 0
    while np.any(label < 0):
        rounds += 1
        todo = np.flatnonzero(label < 0)
        tgt, dist = nearest_open(P[todo], C, count < hi)
        for c in np.unique(tgt):
            mine = np.flatnonzero(tgt == c)
            room = hi - count[c]
            # proposers in (distance, point index) order; todo is increasing
            order = np.lexsort((todo[mine], dist[mine]))
            take = todo[mine[order[:room]]]
            label[take] = c
            count[c] += take.size
    for c in range(k):
        if count[c] >= lo:
            continue
        dc = okm.sqdist_to(P, C[c])
        while count[c] < lo:
            ok = (label != c) & (count[np.maximum(label, 0)] > lo)
            cand = np.flatnonzero(ok)
            i = cand[np.lexsort((cand, dc[cand]))[0]]
            count[label[i]] -= 1
            label[i] = c
            count[c] += 1
    return label.astype(np.int32), rounds


def stable_block_perm(blk, M):
    """Indices sorted by block, points of one block in index order; block_ptr."""
    perm = np.argsort(blk, kind="stable").astype(np.int64)
    ptr = np.r_[0, np.cumsum(np.bincount(blk, minlength=M))].astype(np.int64)
    return perm, ptr


def partition(X, M, lo, hi, iters, rand, U=None):
    """Steps 1-7 above.  Returns a dict with perm, block_ptr (training),
    u_perm, u_block_ptr (test, if U is given), the seeded and Lloyd centres,
    the bounded labels, the block centres in block order, and the chain."""
    X = np.asarray(X, dtype=np.float64)
    C0, seed_idx = seed(X, M, rand)
    C, _, _ = okm.lloyd(X, C0, iters)
    label, rounds = bounded_assign(X, C, lo, hi)
    Cb, count = okm.update(X, label, C)
    chain = okm.chain_order(Cb)
    rank = np.empty(M, dtype=np.int64)
    rank[chain] = np.arange(M)
    perm, ptr = stable_block_perm(rank[label], M)
    out = dict(perm=perm, block_ptr=ptr, seed_idx=seed_idx, C_seed=C0, C_lloyd=C, label=label,
               rounds=rounds, C_blocks=Cb[chain], chain=chain, count=count)
    if U is not None:
        ulab, _ = okm.assign(U, Cb)
        out["u_perm"], out["u_block_ptr"] = stable_block_perm(rank[ulab], M)
        out["u_label"] = ulab
    return out
