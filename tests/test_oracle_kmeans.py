"""Pins for the k-means oracle: each check ties it to an independent
computation (norms from numpy.linalg, scipy's vector quantisation, group means
from numpy) or to a property of Lloyd's iteration (known clusters, fixed
points, a non-increasing objective, ties to the lowest index)."""
import numpy as np
import pytest
from scipy.cluster.vq import vq

from oracle import kmeans as okm


def blobs(seed, k=3, per=200, d=2, spread=0.05):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, 10, size=(k, d))
    X = np.vstack([centres[j] + spread * rng.standard_normal((per, d)) for j in range(k)])
    truth = np.repeat(np.arange(k), per)
    perm = rng.permutation(X.shape[0])
    return X[perm], truth[perm]


@pytest.mark.parametrize("n,d,k", [(500, 3, 7), (300, 1, 4), (200, 12, 30)])
def test_assign_against_norms_and_vq(n, d, k):
    rng = np.random.default_rng(n + d + k)
    P, C = rng.standard_normal((n, d)), rng.standard_normal((k, d))
    lab, dist2 = okm.assign(P, C)
    D = np.linalg.norm(P[:, None, :] - C[None, :, :], axis=2) ** 2
    srt = np.sort(D, axis=1)
    clear = srt[:, 1] - srt[:, 0] > 1e-9 * srt[:, 1] if k > 1 else np.ones(n, bool)
    assert np.array_equal(lab[clear], np.argmin(D, axis=1)[clear])
    assert np.allclose(dist2, D[np.arange(n), lab], rtol=1e-12, atol=0)
    code, _ = vq(P, C)
    assert np.array_equal(lab[clear], code[clear])


def test_ties_go_to_the_lowest_index():
    C = np.array([[1.0, 0.0], [-1.0, 0.0], [1.0, 0.0], [0.0, 5.0]])
    P = np.array([[0.0, 0.0], [1.0, 0.0], [0.9, 0.1], [-3.0, 0.0]])
    lab, dist2 = okm.assign(P, C)
    # (0,0) is at distance 1 from centres 0, 1 and 2; (1,0) and (0.9,0.1) sit on
    # the duplicated centres 0 and 2
    assert lab.tolist() == [0, 0, 0, 1]
    assert dist2[0] == 1.0 and dist2[1] == 0.0


def test_update_is_the_group_mean_and_keeps_empty_centres():
    rng = np.random.default_rng(5)
    P = rng.standard_normal((400, 4))
    lab = rng.integers(0, 6, size=400)
    lab[lab == 3] = 2                      # centre 3 gets no points
    C0 = rng.standard_normal((6, 4))
    C, count = okm.update(P, lab, C0)
    assert np.array_equal(count, np.bincount(lab, minlength=6))
    for c in range(6):
        if count[c]:
            assert np.allclose(C[c], P[lab == c].mean(axis=0), rtol=1e-14, atol=1e-15)
        else:
            assert np.array_equal(C[c], C0[c])


def test_lloyd_recovers_separated_clusters_and_stops_there():
    X, truth = blobs(7)
    first = np.array([np.flatnonzero(truth == j)[0] for j in range(3)])
    C, lab, _ = okm.lloyd(X, X[first], 5)
    assert np.array_equal(lab, truth)
    for j in range(3):
        assert np.allclose(C[j], X[truth == j].mean(axis=0), rtol=1e-14)
    C2, lab2, _ = okm.lloyd(X, C, 1)
    assert np.array_equal(C2, C) and np.array_equal(lab2, lab)


def test_lloyd_objective_does_not_increase():
    rng = np.random.default_rng(11)
    X = rng.uniform(0, 1, size=(800, 3))
    C = X[rng.choice(800, 12, replace=False)]
    prev = np.inf
    for _ in range(8):
        lab, dist2 = okm.assign(X, C)
        obj = dist2.sum()
        assert obj <= prev * (1 + 1e-12)
        prev = obj
        C, _ = okm.update(X, lab, C)


def test_update_is_the_sequential_sum_in_index_order():
    """10000 points: each centre is its points' coordinates added one at a time
    in increasing index from 0, divided once by the count (checked against a
    plain Python loop for a few coordinates), and equals numpy's group mean
    within rounding."""
    rng = np.random.default_rng(3)
    P = rng.standard_normal((10000, 3))
    lab = rng.integers(0, 5, 10000)
    C, _ = okm.update(P, lab, np.zeros((5, 3)))
    for c in range(5):
        assert np.allclose(C[c], P[lab == c].mean(axis=0), rtol=1e-12, atol=1e-15)
    for c, t in ((0, 0), (3, 2)):
        seq = 0.0
        for v in P[lab == c, t]:
            seq = seq + float(v)
        assert C[c, t] == seq / float(np.sum(lab == c))


def test_chain_order_on_a_line_and_visits_every_centre():
    """Centres on a line: the chain starts at the end farther from the mean and
    walks them in sorted order; random centres: a permutation."""
    xs = np.array([0.0, 0.5, 0.6, 2.0, 3.1, 3.3, 7.0])
    perm = np.random.default_rng(2).permutation(xs.size)
    C = np.c_[xs[perm], 2.0 * xs[perm]]
    order = okm.chain_order(C)
    assert np.array_equal(C[order, 0], xs[::-1])     # 7.0 is farthest from the mean 2.5
    R = np.random.default_rng(4).uniform(size=(50, 5))
    assert sorted(okm.chain_order(R).tolist()) == list(range(50))


def test_chain_order_greedy_step_against_brute_force():
    rng = np.random.default_rng(6)
    C = rng.uniform(size=(40, 3))
    order = okm.chain_order(C)
    D = np.linalg.norm(C[:, None] - C[None], axis=2)
    assert order[0] == np.argmax(np.linalg.norm(C - C.mean(0), axis=1))
    for a, b in zip(order[:-1], order[1:]):
        rest = [c for c in range(40) if c not in order[:list(order).index(b)]]
        assert D[a, b] <= D[a, rest].min() * (1 + 1e-12)
