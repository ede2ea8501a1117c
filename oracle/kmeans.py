"""k-means steps of the block partitioner, written out plainly (oracle; test
infrastructure only).

LMA partitions the inputs into M blocks by clustering (section
"Low-Rank-cum-Markov Approximation"; the scheme itself is left to earlier
work).  These are the two steps of Lloyd's iteration, in the evaluation order
that the library's C ABI fixes:

  squared distance  sum over t = 0..d-1, in that order, of (p_t - c_t)^2, each
                    difference, product and sum rounded separately;
  nearest centre    the smallest distance, ties to the lowest centre index
                    (a point whose distances are all NaN keeps centre 0 and
                    distance +inf);
  centre update     the sum, in increasing point index and starting from 0, of
                    the coordinates of the points with that label, divided
                    once by their count; a centre without points keeps its
                    coordinates.

numpy evaluates every elementwise operation below with one rounding and no
fused multiply-add, and cumsum adds in index order.
"""
import numpy as np


def sqdist_to(P, c):
    """Squared distances of all rows of P to one centre c, summed over the
    coordinates in increasing order."""
    acc = np.zeros(P.shape[0])
    for t in range(P.shape[1]):
        df = P[:, t] - c[t]
        acc = acc + df * df
    return acc


def assign(P, C):
    """Nearest centre and its squared distance for every row of P."""
    P, C = np.asarray(P, dtype=np.float64), np.asarray(C, dtype=np.float64)
    best = np.full(P.shape[0], np.inf)
    arg = np.zeros(P.shape[0], dtype=np.int32)
    for c in range(C.shape[0]):
        acc = sqdist_to(P, C[c])
        better = acc < best          # strict: an equal later centre does not win
        best[better] = acc[better]
        arg[better] = c
    return arg, best


def update(P, label, C):
    """New centres (mean of each label's points) and the count per centre."""
    P, C = np.asarray(P, dtype=np.float64), np.array(C, dtype=np.float64)
    label = np.asarray(label)
    count = np.zeros(C.shape[0], dtype=np.int64)
    for c in range(C.shape[0]):
        idx = np.flatnonzero(label == c)
        count[c] = idx.size
        if idx.size == 0:
            continue
        for t in range(P.shape[1]):
            s = np.cumsum(np.r_[0.0, P[idx, t]])[-1]
            C[c, t] = s / float(idx.size)
    return C, count


def lloyd(P, C0, iters):
    """iters rounds of (assign, update) from C0, then the final assignment."""
    C = np.array(C0, dtype=np.float64)
    for _ in range(iters):
        label, _ = assign(P, C)
        C, _ = update(P, label, C)
    label, dist2 = assign(P, C)
    return C, label, dist2
