"""Seeded synthetic inputs for LMA Gaussian-process regression.

This module draws inputs only.  It holds none of the LMA arithmetic: no
covariance function, no low-rank or Markov approximation, no solve.  Both the
CPU oracle and the GPU library consume the arrays it returns, so that the two
sides see identical bytes.

What it draws (each step with its own seeded stream):
  * training inputs X (uniform box or a Gaussian mixture),
  * an approximate GP draw for the outputs by random Fourier features
    (f(x) = sqrt(2 sf2 / F) * sum_j cos(w_j . x + phi_j), w_j ~ N(0, diag(l^-2))),
    plus Gaussian observation noise,
  * a partition of D into M blocks (sort on the first coordinate, or a
    capacity-bounded k-means whose blocks are ordered along a greedy
    nearest-centroid chain so that neighbouring blocks are correlated),
  * the support set S (random rows of X),
  * test inputs U, assigned to test blocks by the same partition rule and
    stored block-contiguously.

The partition is an input of the method (the paper partitions D and U so that
outputs inside a block are as correlated as possible, using a clustering
scheme it does not describe); the chain order of the blocks fixes which
blocks are "next" for the Markov band.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass
from typing import Optional

import numpy as np

ROOT_SEED = 14114510


@dataclass
class Problem:
    """One LMA regression problem, laid out the way the C ABI consumes it."""

    X: np.ndarray                 # [n, d] float64, rows of block m are block_ptr[m]..block_ptr[m+1]-1
    y: np.ndarray                 # [n] float64
    block_ptr: np.ndarray         # [M+1] int64
    S: np.ndarray                 # [s, d] float64 support set
    B: int                        # Markov order
    log_hyp: np.ndarray           # [d+2]: log l_1..log l_d, log sigma_s^2, log sigma_n^2
    prior_mean: float = 0.0
    U: Optional[np.ndarray] = None            # [n_u, d] test inputs, block-contiguous
    u_block_ptr: Optional[np.ndarray] = None  # [M+1] int64
    y_u: Optional[np.ndarray] = None          # noisy test outputs (RMSE only)
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])

    @property
    def s(self) -> int:
        return int(self.S.shape[0])

    @property
    def M(self) -> int:
        return int(len(self.block_ptr) - 1)

    @property
    def n_u(self) -> int:
        return 0 if self.U is None else int(self.U.shape[0])

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)

    def digest(self) -> dict:
        """Checksums that identify the drawn inputs (for stored expected values)."""
        out = {
            "n": self.n, "d": self.d, "s": self.s, "M": self.M, "B": int(self.B),
            "n_u": self.n_u,
            "block_ptr_sum": int(np.sum(self.block_ptr * np.arange(1, self.M + 2))),
            "X_sum": float(np.sum(self.X)), "y_sum": float(np.sum(self.y)),
            "S_sum": float(np.sum(self.S)),
        }
        if self.U is not None:
            out["u_block_ptr_sum"] = int(np.sum(self.u_block_ptr * np.arange(1, self.M + 2)))
            out["U_sum"] = float(np.sum(self.U))
        return out


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def _streams(seed, k: int):
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(k)]


def rff_draw(rng: np.random.Generator, point_sets, ell, sf2: float, F: int,
             chunk: int = 4096):
    """Approximate zero-mean GP draw by F random Fourier features.

    Returns one array of function values per entry of `point_sets`; the same
    features are used for all sets, so the draws are jointly consistent.
    """
    point_sets = list(point_sets)
    d = point_sets[0].shape[1]
    ell = np.broadcast_to(np.asarray(ell, dtype=np.float64), (d,))
    W = rng.standard_normal((F, d)) / ell[None, :]
    phi = rng.uniform(0.0, 2.0 * np.pi, size=F)
    amp = np.sqrt(2.0 * sf2 / F)
    outs = []
    for P in point_sets:
        f = np.empty(P.shape[0])
        for a in range(0, P.shape[0], chunk):
            Z = P[a:a + chunk] @ W.T
            Z += phi[None, :]
            np.cos(Z, out=Z)
            f[a:a + chunk] = amp * Z.sum(axis=1)
        outs.append(f)
    return outs


def _sqdist(P, C):
    """Squared Euclidean distances between rows of P and rows of C (for clustering)."""
    d2 = (P * P).sum(1)[:, None] - 2.0 * (P @ C.T) + (C * C).sum(1)[None, :]
    np.maximum(d2, 0.0, out=d2)
    return d2


def _kmeanspp(rng, P, k):
    n = P.shape[0]
    centres = np.empty((k, P.shape[1]))
    centres[0] = P[rng.integers(n)]
    dmin = ((P - centres[0]) ** 2).sum(1)
    for i in range(1, k):
        prob = dmin / dmin.sum()
        centres[i] = P[rng.choice(n, p=prob)]
        dmin = np.minimum(dmin, ((P - centres[i]) ** 2).sum(1))
    return centres


def _lloyd(P, centres, iters):
    k = centres.shape[0]
    for _ in range(iters):
        lab = np.argmin(_sqdist(P, centres), axis=1)
        cnt = np.bincount(lab, minlength=k)
        new = np.zeros_like(centres)
        for j in range(P.shape[1]):
            new[:, j] = np.bincount(lab, weights=P[:, j], minlength=k)
        live = cnt > 0
        centres = centres.copy()
        centres[live] = new[live] / cnt[live, None]
    return centres


def _capacity_assign(D2, lo: int, hi: int):
    """Greedy capacity-bounded assignment: every cluster ends with lo..hi points.

    Points whose nearest centre is clearly better than their second choice are
    placed first; a point whose preferred centres are full falls through to
    the next nearest one.  Clusters left below `lo` then take the closest
    points from clusters that can spare them.
    """
    n, k = D2.shape
    assert lo * k <= n <= hi * k, "capacities cannot be met"
    K = min(k, 16)
    near = np.argpartition(D2, K - 1, axis=1)[:, :K]
    dn = np.take_along_axis(D2, near, axis=1)
    o = np.argsort(dn, axis=1, kind="stable")
    near = np.take_along_axis(near, o, axis=1)
    dn = np.take_along_axis(dn, o, axis=1)
    margin = dn[:, 1] - dn[:, 0] if K > 1 else np.zeros(n)
    order = np.argsort(-margin, kind="stable")
    assign = np.full(n, -1, dtype=np.int64)
    counts = np.zeros(k, dtype=np.int64)
    for r in range(K):
        pending = order[assign[order] < 0]
        if pending.size == 0:
            break
        cand = near[pending, r]
        idx = np.argsort(cand, kind="stable")
        cs = cand[idx]
        starts = np.r_[0, np.flatnonzero(cs[1:] != cs[:-1]) + 1]
        lens = np.diff(np.r_[starts, cs.size])
        rank = np.arange(cs.size) - np.repeat(starts, lens)
        ok = rank < (hi - counts[cs])
        assign[pending[idx[ok]]] = cs[ok]
        counts += np.bincount(cs[ok], minlength=k)
    for p in order[assign[order] < 0]:
        for c in np.argsort(D2[p], kind="stable"):
            if counts[c] < hi:
                assign[p] = c
                counts[c] += 1
                break
    for c in np.flatnonzero(counts < lo):
        for p in np.argsort(D2[:, c], kind="stable"):
            if counts[c] >= lo:
                break
            o_c = assign[p]
            if o_c != c and counts[o_c] > lo:
                assign[p] = c
                counts[o_c] -= 1
                counts[c] += 1
    assert counts.min() >= lo and counts.max() <= hi
    return assign


def _chain_order(C):
    """Greedy nearest-neighbour chain through the centres, from the centre with
    the smallest first-principal-component coordinate."""
    k = C.shape[0]
    Cc = C - C.mean(0)
    _, _, vt = np.linalg.svd(Cc, full_matrices=False)
    v = vt[0]
    v = v if v[np.argmax(np.abs(v))] > 0 else -v
    cur = int(np.argmin(Cc @ v))
    seen = np.zeros(k, dtype=bool)
    order = [cur]
    seen[cur] = True
    for _ in range(k - 1):
        dd = ((C - C[cur]) ** 2).sum(1)
        dd[seen] = np.inf
        cur = int(np.argmin(dd))
        order.append(cur)
        seen[cur] = True
    return np.asarray(order)


def kmeans_partition(rng, X, M, lo, hi, iters=20, U=None):
    """Capacity-bounded k-means partition with chain-ordered blocks.

    Returns (perm, block_ptr, uperm, u_block_ptr): X[perm] is block-contiguous,
    U[uperm] is block-contiguous with test points assigned to the nearest
    block centre."""
    n = X.shape[0]
    # centres from subsamples (k-means++ seeding, then Lloyd), assignment of all points
    sub_pp = X[np.sort(rng.choice(n, size=min(n, 64 * M), replace=False))] if n > 64 * M else X
    sub_ll = X[np.sort(rng.choice(n, size=min(n, 512 * M), replace=False))] if n > 512 * M else X
    C = _lloyd(sub_ll, _kmeanspp(rng, sub_pp, M), iters)
    lab = _capacity_assign(_sqdist(X, C), lo, hi)
    cnt = np.bincount(lab, minlength=M)
    Cf = np.zeros_like(C)
    for j in range(X.shape[1]):
        Cf[:, j] = np.bincount(lab, weights=X[:, j], minlength=M) / cnt
    chain = _chain_order(Cf)
    rank = np.empty(M, dtype=np.int64)
    rank[chain] = np.arange(M)
    blk = rank[lab]
    perm = np.argsort(blk, kind="stable")
    block_ptr = np.r_[0, np.cumsum(np.bincount(blk, minlength=M))].astype(np.int64)
    if U is None:
        return perm, block_ptr, None, None
    ublk = rank[np.argmin(_sqdist(U, Cf), axis=1)]
    uperm = np.argsort(ublk, kind="stable")
    u_block_ptr = np.r_[0, np.cumsum(np.bincount(ublk, minlength=M))].astype(np.int64)
    return perm, block_ptr, uperm, u_block_ptr


def sorted_partition(X, sizes, U=None):
    """Partition by sorting on the first coordinate into blocks of the given
    sizes; test points go to the block whose x1-interval contains them (the
    interval boundaries are midpoints between neighbouring blocks)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    perm = np.argsort(X[:, 0], kind="stable")
    block_ptr = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    if U is None:
        return perm, block_ptr, None, None
    xs = X[perm, 0]
    cuts = 0.5 * (xs[block_ptr[1:-1] - 1] + xs[block_ptr[1:-1]])
    ublk = np.searchsorted(cuts, U[:, 0], side="right")
    uperm = np.argsort(ublk, kind="stable")
    M = len(sizes)
    u_block_ptr = np.r_[0, np.cumsum(np.bincount(ublk, minlength=M))].astype(np.int64)
    return perm, block_ptr, uperm, u_block_ptr


def _loguniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def make_random(seed=0, n=200, d=2, M=6, s=12, n_u=40, B=1, uneven=(17, 40),
                empty_test_block=None, ell_range=(0.2, 0.8), sf2=1.0, sn2=0.05,
                prior_mean=0.0, s_from_X=True, F=1024, name="random"):
    """Small problem with uneven blocks, for oracle pins and parity tests.

    Blocks come from sorting on x1; block sizes are drawn in `uneven`
    (then rescaled to sum to n).  `empty_test_block` removes the test points
    that fall into that block, so its test block is empty."""
    r_x, r_f, r_e, r_s, r_u, r_p = _streams(seed, 6)
    raw = r_p.integers(uneven[0], uneven[1] + 1, size=M).astype(np.float64)
    sizes = np.maximum(1, np.floor(raw / raw.sum() * n)).astype(np.int64)
    sizes[-1] += n - sizes.sum()
    assert sizes.min() >= 1
    X0 = r_x.uniform(0.0, 1.0, size=(n, d))
    U0 = r_u.uniform(0.0, 1.0, size=(n_u, d)) if n_u > 0 else None
    ell = _loguniform(r_p, ell_range[0], ell_range[1], size=d)
    perm, bp, uperm, ubp = sorted_partition(X0, sizes, U0)
    X = X0[perm]
    U = None if U0 is None else U0[uperm]
    if U is not None and empty_test_block is not None:
        q = int(empty_test_block)
        keep = np.ones(U.shape[0], dtype=bool)
        keep[ubp[q]:ubp[q + 1]] = False
        cnt = np.diff(ubp)
        cnt[q] = 0
        U = U[keep]
        ubp = np.r_[0, np.cumsum(cnt)].astype(np.int64)
    sets = [X] + ([U] if U is not None else [])
    fs = rff_draw(r_f, sets, ell, sf2, F)
    y = prior_mean + fs[0] + np.sqrt(sn2) * r_e.standard_normal(n)
    y_u = None
    if U is not None:
        y_u = prior_mean + fs[1] + np.sqrt(sn2) * r_e.standard_normal(U.shape[0])
    if s_from_X:
        S = X[np.sort(r_s.choice(n, size=s, replace=False))].copy()
    else:
        S = r_s.uniform(0.0, 1.0, size=(s, d))
    log_hyp = np.r_[np.log(ell), np.log(sf2), np.log(sn2)]
    return Problem(X=X, y=y, block_ptr=bp, S=S, B=int(B), log_hyp=log_hyp,
                   prior_mean=float(prior_mean), U=U, u_block_ptr=ubp, y_u=y_u,
                   name=name)


def config_seed(k: int):
    return np.random.SeedSequence(ROOT_SEED).spawn(5)[k]


def make_config0(F=8192):
    """n=2048 in [0,1]^4, l_i ~ logU[0.1,1], sf2=1, sn2=0.01; M=8 blocks of
    256 by x1, B=1, |S|=64 rows of X, 256 test points by x1 interval."""
    r_x, r_f, r_e, r_s, r_u, r_p = _streams(config_seed(0), 6)
    n, d, M, s, n_u = 2048, 4, 8, 64, 256
    ell = _loguniform(r_p, 0.1, 1.0, size=d)
    sf2, sn2 = 1.0, 0.01
    X0 = r_x.uniform(0, 1, size=(n, d))
    U0 = r_u.uniform(0, 1, size=(n_u, d))
    perm, bp, uperm, ubp = sorted_partition(X0, [n // M] * M, U0)
    X, U = X0[perm], U0[uperm]
    f, fu = rff_draw(r_f, [X, U], ell, sf2, F)
    y = f + np.sqrt(sn2) * r_e.standard_normal(n)
    y_u = fu + np.sqrt(sn2) * r_e.standard_normal(n_u)
    S = X[np.sort(r_s.choice(n, size=s, replace=False))].copy()
    return Problem(X=X, y=y, block_ptr=bp, S=S, B=1,
                   log_hyp=np.r_[np.log(ell), np.log(sf2), np.log(sn2)],
                   U=U, u_block_ptr=ubp, y_u=y_u, name="cfg0")


def make_uniform_kmeans(k, n, d, M, B, s, n_u, sn2, F=4096, name=""):
    r_x, r_f, r_e, r_s, r_u, r_p = _streams(config_seed(k), 6)
    ell = _loguniform(r_p, 0.1, 1.0, size=d)
    sf2 = 1.0
    X0 = r_x.uniform(0, 1, size=(n, d))
    U0 = r_u.uniform(0, 1, size=(n_u, d)) if n_u else None
    b = n // M
    perm, bp, uperm, ubp = kmeans_partition(r_p, X0, M, b, b, U=U0)
    X = X0[perm]
    U = None if U0 is None else U0[uperm]
    sets = [X] + ([U] if U is not None else [])
    fs = rff_draw(r_f, sets, ell, sf2, F)
    y = fs[0] + np.sqrt(sn2) * r_e.standard_normal(n)
    y_u = None if U is None else fs[1] + np.sqrt(sn2) * r_e.standard_normal(n_u)
    S = X[np.sort(r_s.choice(n, size=s, replace=False))].copy()
    return Problem(X=X, y=y, block_ptr=bp, S=S, B=B,
                   log_hyp=np.r_[np.log(ell), np.log(sf2), np.log(sn2)],
                   U=U, u_block_ptr=ubp, y_u=y_u, name=name)


def make_config1(F=4096):
    """n=65536 in [0,1]^8, sn2=0.05; M=64 k-means blocks of 1024, B=2,
    |S|=512, 8192 test points by nearest block centre."""
    return make_uniform_kmeans(1, 65536, 8, 64, 2, 512, 8192, 0.05, F=F, name="cfg1")


def make_config3(F=4096):
    """As the n=65536 workload but n=131072, M=128 blocks of 1024, no test set
    (log marginal likelihood and its gradient)."""
    return make_uniform_kmeans(3, 131072, 8, 128, 2, 512, 0, 0.05, F=F, name="cfg3")


def make_config2(F=512, n=524288, M=256, n_u=65536, s=1024, B=3, sn2_model=0.01,
                 lo=1024, hi=3072, kmeans_iters=10):
    """n=524288 in 21-D drawn from an equal-weight mixture of 32 Gaussians
    (centres ~ U[0,1]^21, spread N(0, 0.2^2 I)); outputs = smooth RFF draw
    (l=1, sf2=1) + rough RFF draw (l=0.05, sf2=1) + noise of variance 0.01.
    M=256 k-means blocks with sizes bounded to [1024, 3072], chain-ordered,
    B=3, |S|=1024 rows of X, 65536 test points from the same mixture.
    Model hyperparameters: l_i=1, sf2=1, sn2=`sn2_model`."""
    d = 21
    r_x, r_f, r_e, r_s, r_u, r_p = _streams(config_seed(2), 6)
    centres = r_x.uniform(0, 1, size=(32, d))
    X0 = centres[r_x.integers(32, size=n)] + 0.2 * r_x.standard_normal((n, d))
    U0 = centres[r_u.integers(32, size=n_u)] + 0.2 * r_u.standard_normal((n_u, d))
    perm, bp, uperm, ubp = kmeans_partition(r_p, X0, M, lo, hi, iters=kmeans_iters, U=U0)
    X, U = X0[perm], U0[uperm]
    fs1, fu1 = rff_draw(r_f, [X, U], 1.0, 1.0, F)
    fs2, fu2 = rff_draw(r_f, [X, U], 0.05, 1.0, F)
    y = fs1 + fs2 + 0.1 * r_e.standard_normal(n)
    y_u = fu1 + fu2 + 0.1 * r_e.standard_normal(n_u)
    S = X[np.sort(r_s.choice(n, size=s, replace=False))].copy()
    log_hyp = np.r_[np.zeros(d), 0.0, np.log(sn2_model)]
    return Problem(X=X, y=y, block_ptr=bp, S=S, B=B, log_hyp=log_hyp,
                   U=U, u_block_ptr=ubp, y_u=y_u, name="cfg2")


SUPPORT_SEED = 20150125


def nested_support(X, s, seed=SUPPORT_SEED):
    """Support set of the |S| x B sweep: the first s rows (in index order) of
    one seeded permutation of the training points, so that smaller support
    sets are subsets of larger ones."""
    order = np.random.default_rng(seed).permutation(X.shape[0])
    return X[np.sort(order[:s])].copy()


def make_sweep16k(s, B):
    """The n=16384 workload of the |S| x B sweep: X ~ U[0,1]^8, GP-sample
    outputs (l_i ~ logU[0.1, 1], sf2=1, sn2=0.05), M=16 k-means blocks of 1024,
    4096 test points; support set of size s from nested_support; Markov order
    B (B = 15 = M-1 is the full GP)."""
    p = make_uniform_kmeans(1, 16384, 8, 16, B, 16, 4096, 0.05, name=f"n16384_S{s}_B{B}")
    return p.with_(S=nested_support(p.X, s))


def make_config(k: int, **kw) -> Problem:
    return {0: make_config0, 1: make_config1, 2: make_config2, 3: make_config3}[k](**kw)


def default_theta0(y, d):
    """Default start for hyperparameter fitting: l_i = 1, sf2 = Var(y),
    sn2 = 0.1 Var(y)."""
    v = float(np.var(y))
    return np.r_[np.zeros(d), np.log(v), np.log(0.1 * v)]
