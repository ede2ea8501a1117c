"""Pins for the CPU oracle: each check ties the oracle to something other than
itself (a textbook GP computed by library routines, the PIC special case, the
structural results of Proposition 1, Theorem 1 and Lemma 1, finite
differences).  A plausible slip in the oracle (a wrong neighbour set, a
dropped term, a transposed block) fails at least one of them."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.stats import multivariate_normal

import synth
from oracle import dense, lma, summaries
from oracle.covariance import k_cross, k_same

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def tiny(seed=3, **kw):
    base = dict(n=180, d=2, M=6, s=12, n_u=40, B=1, empty_test_block=2)
    base.update(kw)
    return synth.make_random(seed=seed, **base)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


# --- limits stated in the paper --------------------------------------------

def textbook_gp(p):
    """Full GP regression (Section "Full-Rank Gaussian Process Regression"),
    with the SE-ARD covariance and noise on the diagonal of D and of U."""
    Sdd = k_same(p.X, p.log_hyp)
    Sud = k_cross(p.U, p.X, p.log_hyp)
    F = sla.cho_factor(Sdd, lower=True)
    c = p.y - p.prior_mean
    mean = p.prior_mean + Sud @ sla.cho_solve(F, c)
    sf2, sn2 = np.exp(p.log_hyp[-2]), np.exp(p.log_hyp[-1])
    var = sf2 + sn2 - np.einsum("ij,ji->i", Sud, sla.cho_solve(F, Sud.T))
    lml = multivariate_normal(mean=np.full(p.n, p.prior_mean), cov=Sdd).logpdf(p.y)
    return mean, var, lml


@pytest.mark.parametrize("seed", [1, 3])
def test_full_gp_at_maximal_order(seed):
    """B = M-1 makes Sigma_bar equal Sigma, so LMA is the full GP."""
    p = tiny(seed, prior_mean=0.3)
    q = p.with_(B=p.M - 1)
    mean, var, lml = textbook_gp(q)
    m0, v0 = dense.predict(q)
    assert rel(m0, mean) < 1e-11 and rel(v0, var) < 1e-11
    assert abs(dense.lml(q) - lml) < 1e-9 * abs(lml)
    r = lma.fit_predict(q)
    assert rel(r["mean"], mean) < 1e-11 and rel(r["var"], var) < 1e-11
    assert abs(r["lml"] - lml) < 1e-9 * abs(lml)


def test_pic_at_order_zero():
    """B = 0 gives the PIC prior: Q over V plus the exact residual inside each
    block V_m = D_m u U_m and zero residual across blocks."""
    p = tiny(5).with_(B=0)
    P = np.vstack([p.X, p.U])
    Sig = k_same(P, p.log_hyp)
    Kvs = k_cross(P, p.S, p.log_hyp)
    Q = Kvs @ np.linalg.solve(k_same(p.S, p.log_hyp), Kvs.T)
    R = Sig - Q
    bp, ubp, n = p.block_ptr, p.u_block_ptr, p.n
    blk = np.empty(P.shape[0], dtype=int)
    for m in range(p.M):
        blk[bp[m]:bp[m + 1]] = m
        blk[n + ubp[m]:n + ubp[m + 1]] = m
    Spic = Q + R * (blk[:, None] == blk[None, :])
    D, U = np.arange(n), n + np.arange(p.n_u)
    F = sla.cho_factor(Spic[np.ix_(D, D)], lower=True)
    mean = Spic[np.ix_(U, D)] @ sla.cho_solve(F, p.y)
    var = np.diag(Spic[np.ix_(U, U)] - Spic[np.ix_(U, D)] @ sla.cho_solve(F, Spic[np.ix_(D, U)]))
    m0, v0 = dense.predict(p)
    assert rel(m0, mean) < 1e-11 and rel(v0, var) < 1e-11
    r = lma.fit_predict(p)
    assert rel(r["mean"], mean) < 1e-11 and rel(r["var"], var) < 1e-11
    lml = multivariate_normal(mean=np.zeros(n), cov=Spic[np.ix_(D, D)]).logpdf(p.y)
    assert abs(r["lml"] - lml) < 1e-9 * abs(lml)


def test_intermediate_order_differs_from_both_limits():
    """0 < B < M-1 is neither PIC nor the full GP (guards against a recursion
    that silently returns one of the limits)."""
    p = tiny(7).with_(B=2)
    m_b, _ = dense.predict(p)
    m_pic, _ = dense.predict(p.with_(B=0))
    m_fgp, _ = dense.predict(p.with_(B=p.M - 1))
    assert rel(m_b, m_pic) > 1e-6 and rel(m_b, m_fgp) > 1e-6


# --- structure of R_bar ------------------------------------------------------

def band_mask(dn, B):
    n = dn.n
    blk = np.empty(n, dtype=int)
    for m in range(dn.M):
        blk[dn.Didx[m]] = m
    return np.abs(blk[:, None] - blk[None, :]) <= B


@pytest.mark.parametrize("B", [1, 2, 3])
def test_rbar_inverse_is_block_banded(B):
    """Proposition 1: blocks of R_bar_DD^-1 outside the B-band are zero."""
    dn = dense.Dense(tiny(11).with_(B=B))
    D = dn.D
    Ri = np.linalg.inv(dn.Rbar[np.ix_(D, D)])
    off = Ri[~band_mask(dn, B)]
    assert np.abs(off).max() < 1e-9 * np.abs(Ri).max()
    # and the band itself is not trivially zero
    assert np.abs(Ri[band_mask(dn, B) & ~band_mask(dn, 0)]).max() > 1e-3 * np.abs(Ri).max()


@pytest.mark.parametrize("B", [1, 2])
def test_rbar_symmetric_and_matches_band(B):
    """R_bar is symmetric (its upper and lower off-band cases agree) and equals
    R inside the band."""
    dn = dense.Dense(tiny(13).with_(B=B))
    assert np.abs(dn.Rbar - dn.Rbar.T).max() < 1e-12 * np.abs(dn.Rbar).max()
    D = dn.D
    mask = band_mask(dn, B)
    assert np.abs((dn.Rbar[np.ix_(D, D)] - dn.R[np.ix_(D, D)])[mask]).max() == 0.0


def kl(R, Rh):
    n = R.shape[0]
    A = np.linalg.solve(Rh, R)
    return 0.5 * (np.trace(A) - np.linalg.slogdet(A)[1] - n)


@pytest.mark.parametrize("B", [1, 2])
def test_theorem1_kl_optimality(B):
    """Theorem 1: tr(R R_bar^-1) = |D|, and for any R_hat whose inverse is
    B-block-banded, KL(R, R_hat) = KL(R, R_bar) + KL(R_bar, R_hat) >= KL(R, R_bar)."""
    dn = dense.Dense(tiny(17).with_(B=B))
    D = dn.D
    R, Rb = dn.R[np.ix_(D, D)], dn.Rbar[np.ix_(D, D)]
    assert abs(np.trace(np.linalg.solve(Rb, R)) - dn.n) < 1e-8 * dn.n
    rng = np.random.default_rng(0)
    mask = band_mask(dn, B)
    base = kl(R, Rb)
    for t in range(3):
        # random SPD matrix with B-block-banded inverse: P = A A^T restricted to the band, made SPD
        A = rng.standard_normal((dn.n, dn.n)) * mask
        P = A @ A.T * mask + dn.n * np.eye(dn.n)
        Rh = np.linalg.inv(P)
        k1 = kl(R, Rh)
        assert k1 >= base - 1e-9
        assert abs(k1 - (base + kl(Rb, Rh))) < 1e-7 * max(1.0, k1)


@pytest.mark.parametrize("B", [1, 2])
def test_lemma1_banded_cholesky(B):
    """Lemma 1: the upper Cholesky factor U of R_bar_DD^-1 is zero outside the
    B-band, U_mm is the Cholesky factor of Rdot_m and U^B_m = -U_mm R'_m, with
    Rdot_m and R'_m as in Definition 1."""
    dn = dense.Dense(tiny(19).with_(B=B))
    D = dn.D
    Ri = np.linalg.inv(dn.Rbar[np.ix_(D, D)])
    Ri = 0.5 * (Ri + Ri.T)
    Uf = np.linalg.cholesky(Ri).T  # R_bar^-1 = U^T U, U upper
    scale = np.abs(Uf).max()
    for m in range(dn.M):
        ls = summaries.local_summary(dn, m)
        Dm = dn.Didx[m]
        Umm = Uf[np.ix_(Dm, Dm)]
        assert np.abs(Umm.T @ Umm - ls["Rdot"]).max() < 1e-7 * np.abs(ls["Rdot"]).max()
        DB = dn.DB(m)
        if DB.size:
            assert np.abs(Uf[np.ix_(Dm, DB)] + Umm @ ls["Rp"]).max() < 1e-7 * scale
        far = np.concatenate([dn.Didx[k] for k in range(dn.M) if k - m > B] or [np.zeros(0, int)])
        if far.size:
            assert np.abs(Uf[np.ix_(Dm, far)]).max() < 1e-9 * scale


# --- routes to the prediction ------------------------------------------------

@pytest.mark.parametrize("B", [0, 1, 2, 3, 5])
def test_theorem2_route_equals_definition(B):
    """Definition 1 + Definition 2 + Theorem 2 give Eqs. (3)-(4)."""
    p = tiny(23, prior_mean=-0.4).with_(B=B)
    m0, v0 = dense.predict(p)
    m1, v1 = summaries.predict(p)
    assert rel(m1, m0) < 1e-10 and rel(v1, v0) < 1e-10


@pytest.mark.parametrize("B", [0, 1, 2, 3, 4, 5, 9])
def test_window_form_equals_definition(B):
    """The whitened-window form (prediction, variance and LML) equals the
    dense definition for every B, with uneven blocks and an empty test block."""
    p = tiny(29, M=7, n=220, prior_mean=0.7, empty_test_block=3).with_(B=B)
    m0, v0 = dense.predict(p)
    l0 = dense.lml(p)
    r = lma.fit_predict(p)
    assert rel(r["mean"], m0) < 1e-10
    assert rel(r["var"], v0) < 1e-10
    assert abs(r["lml"] - l0) < 1e-10 * abs(l0)


def test_window_form_with_support_off_data_and_d4():
    p = synth.make_random(seed=31, n=240, d=4, M=5, s=20, n_u=30, B=2, s_from_X=False)
    m0, v0 = dense.predict(p)
    r = lma.fit_predict(p)
    assert rel(r["mean"], m0) < 1e-10 and rel(r["var"], v0) < 1e-10
    assert abs(r["lml"] - dense.lml(p)) < 1e-10 * abs(dense.lml(p))


def test_variance_below_prior_and_positive():
    """A well-separated case: every variance lies between the noise and the
    prior variance (the upper bound holds always, see below)."""
    p = tiny(37).with_(B=1)
    r = lma.fit_predict(p)
    sf2, sn2 = np.exp(p.log_hyp[-2]), np.exp(p.log_hyp[-1])
    assert np.all(r["var"] > sn2 * (1 - 1e-9)) and np.all(r["var"] <= sf2 + sn2 + 1e-12)


def negvar_case(B):
    return synth.make_random(seed=3, n=600, d=3, M=8, s=6, n_u=300, B=B, uneven=(50, 100),
                             ell_range=(0.1, 0.4), sn2=0.01, name="negvar")


@pytest.mark.parametrize("B", [1, 2])
def test_variance_can_be_negative_between_the_limits(B):
    """Eq. (1) completes the residual over V = D u U with conditioning sets of
    training blocks only, so a test point keeps its exact residual covariance
    with the blocks B before and B after its own while those two blocks are
    joined only through the Markov approximation.  Sigma_bar_DD stays positive
    definite (Theorem 1), so Eq. (4) never exceeds the prior variance, but
    Sigma_bar_VV can be indefinite for 0 < B < M - 1 and then some predictive
    variances of Eq. (4) are negative.  The window form gives the same values;
    at B = 0 (PIC) and B = M - 1 (full GP) the same inputs give a positive
    definite Sigma_bar_VV and positive variances."""
    p = negvar_case(B)
    D = dense.Dense(p)
    m0, v0 = D.predict()
    assert np.linalg.eigvalsh(D.Sbar[:p.n, :p.n]).min() > 0
    assert np.linalg.eigvalsh(D.Sbar).min() < 0
    assert np.sum(v0 < 0) >= 1
    sf2, sn2 = np.exp(p.log_hyp[-2]), np.exp(p.log_hyp[-1])
    assert np.all(v0 <= sf2 + sn2 + 1e-12)
    r = lma.fit_predict(p)
    assert np.max(np.abs(r["var"] - v0)) < 1e-12 and rel(r["mean"], m0) < 1e-12
    for Bl in (0, p.M - 1):
        Dl = dense.Dense(negvar_case(Bl))
        assert np.linalg.eigvalsh(Dl.Sbar).min() > 0
        assert np.all(Dl.predict()[1] > 0)


# --- gradient ---------------------------------------------------------------

def fd5(p, h=1e-3):
    g = np.zeros(p.d + 2)
    for j in range(p.d + 2):
        def f(t):
            e = np.zeros(p.d + 2)
            e[j] = t
            return dense.lml(p.with_(log_hyp=p.log_hyp + e))
        g[j] = (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)
    return g


@pytest.mark.parametrize("B", [0, 1, 2, 5])
def test_lml_adjoint_matches_finite_differences(B):
    p = tiny(41, n=150, M=5, prior_mean=0.2).with_(B=B)
    val, grad = lma.lml_grad(p)
    assert abs(val - dense.lml(p)) < 1e-10 * abs(val)
    fd = fd5(p)
    assert np.abs(grad - fd).max() < 1e-6 * max(1.0, np.abs(fd).max())


# --- full predictive covariance (Eq. (4) beyond the diagonal) --------------

def test_full_covariance_of_the_full_gp_at_maximal_order():
    """B = M-1: the dense definition's and the window form's full predictive
    covariance equal the textbook GP posterior covariance of the noisy
    outputs, computed by library routines."""
    p = tiny(7, prior_mean=-0.2)
    q = p.with_(B=p.M - 1)
    Sdd = k_same(q.X, q.log_hyp)
    Sud = k_cross(q.U, q.X, q.log_hyp)
    ref = k_same(q.U, q.log_hyp) - Sud @ sla.cho_solve(sla.cho_factor(Sdd, lower=True), Sud.T)
    _, c0 = dense.predict(q, full_cov=True)
    _, c1 = lma.predict_cov(q)
    assert rel(c0, ref) < 1e-11 and rel(c1, ref) < 1e-11


def test_full_covariance_of_pic_at_order_zero():
    """B = 0: the full covariance of the PIC prior (exact residual inside each
    V_m = D_m u U_m, none across blocks), conditioned on D directly."""
    p = tiny(5).with_(B=0)
    P = np.vstack([p.X, p.U])
    Sig = k_same(P, p.log_hyp)
    Kvs = k_cross(P, p.S, p.log_hyp)
    Q = Kvs @ np.linalg.solve(k_same(p.S, p.log_hyp), Kvs.T)
    R = Sig - Q
    bp, ubp, n = p.block_ptr, p.u_block_ptr, p.n
    blk = np.empty(P.shape[0], dtype=int)
    for m in range(p.M):
        blk[bp[m]:bp[m + 1]] = m
        blk[n + ubp[m]:n + ubp[m + 1]] = m
    Spic = Q + R * (blk[:, None] == blk[None, :])
    D, U = np.arange(n), n + np.arange(p.n_u)
    F = sla.cho_factor(Spic[np.ix_(D, D)], lower=True)
    ref = Spic[np.ix_(U, U)] - Spic[np.ix_(U, D)] @ sla.cho_solve(F, Spic[np.ix_(D, U)])
    _, c0 = dense.predict(p, full_cov=True)
    _, c1 = lma.predict_cov(p)
    assert rel(c0, ref) < 1e-11 and rel(c1, ref) < 1e-11


@pytest.mark.parametrize("B", [1, 2, 3])
def test_full_covariance_window_form_equals_the_definition(B):
    """0 < B < M-1: the window form (banded residual minus the whitened
    products, plus the low-rank term) equals Eq. (4) of the dense definition
    entry by entry, on uneven blocks with an empty test block and a support
    set off the data; its diagonal is the predictive variance; and pairs of
    test points more than B blocks apart carry only the low-rank term."""
    p = tiny(11, B=B, s_from_X=False, prior_mean=0.1)
    _, c0 = dense.predict(p, full_cov=True)
    f = lma.Fit(p, keep_test_cols=True).finish()
    c1 = f.predict_cov()
    scale = np.max(np.abs(c0))
    assert np.max(np.abs(c1 - c0)) <= 1e-12 * scale
    _, var = f.predict()
    assert np.max(np.abs(np.diag(c1) - var)) <= 1e-13 * scale
    E = f.K_SU.T - f.G
    low = E @ sla.cho_solve((f.L_dd, True), E.T)
    ublk = np.repeat(np.arange(p.M), np.diff(p.u_block_ptr))
    far = np.abs(ublk[:, None] - ublk[None, :]) > B
    assert far.any()
    assert np.max(np.abs(c0[far] - low[far])) <= 1e-12 * scale
    assert np.max(np.abs(c0[~far] - low[~far])) > 1e-6 * scale
