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
  chain order       blocks ordered along the Markov chain: start at the centre
                    farthest from the centres' mean (summed over the centres in
                    index order, divided by k), then move to the nearest centre
                    not yet visited (ties to the lowest index);
  centre update     the mean of the points with that label: their
                    coordinates summed in increasing point index starting from
                    0, then one division by the count; a centre without points
                    keeps its coordinates.  (The library may sum in another
                    order; its result then differs from this one by rounding
                    only, within the bound of the summation error.)

numpy evaluates every elementwise operation below with one rounding and no
fused multiply-add, and cumsum adds in index order (along the given axis).
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
    d = P.shape[1]
    count = np.zeros(C.shape[0], dtype=np.int64)
    for c in range(C.shape[0]):
        rows = P[label == c]
        count[c] = rows.shape[0]
        if count[c] == 0:
            continue
        # sequential sum in increasing index (cumsum adds in order)
        total = np.cumsum(np.vstack([np.zeros((1, d)), rows]), axis=0)[-1]
        C[c] = total / float(count[c])
    return C, count


def lloyd(P, C0, iters):
    """iters rounds of (assign, update) from C0, then the final assignment."""
    C = np.array(C0, dtype=np.float64)
    for _ in range(iters):
        label, _ = assign(P, C)
        C, _ = update(P, label, C)
    label, dist2 = assign(P, C)
    return C, label, dist2


def chain_order(C):
    """Order of the centres along a nearest-neighbour chain from the centre
    farthest from their mean."""
    C = np.asarray(C, dtype=np.float64)
    k = C.shape[0]
    mean = np.cumsum(np.vstack([np.zeros((1, C.shape[1])), C]), axis=0)[-1] / float(k)
    far = sqdist_to(C, mean)
    cur = int(np.argmax(far))        # first index among equal maxima
    seen = np.zeros(k, dtype=bool)
    order = [cur]
    seen[cur] = True
    for _ in range(k - 1):
        dd = sqdist_to(C, C[cur])
        dd[seen] = np.inf
        cur = int(np.argmin(dd))     # first index among equal minima
        order.append(cur)
        seen[cur] = True
    return np.asarray(order, dtype=np.int32)
