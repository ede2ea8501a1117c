"""Dense definition of LMA (oracle tier O0).  Test infrastructure only.

Builds every matrix of the approximation explicitly over V = D u U and applies
the definitions of the section "Low-Rank-cum-Markov Approximation":

  Q_BB' = Sigma_BS Sigma_SS^-1 Sigma_SB'        (low-rank part)
  R_BB' = Sigma_BB' - Q_BB'                      (residual)
  R_bar by the recursion of Eq. (1)
  Sigma_bar = Q + R_bar                          (Eq. (2))
  mean  = mu + Sigma_bar_UD Sigma_bar_DD^-1 (y - mu)          (Eq. (3))
  cov   = Sigma_bar_UU - Sigma_bar_UD Sigma_bar_DD^-1 Sigma_bar_DU   (Eq. (4))
  lml   = log N(y; mu, Sigma_bar_DD)

Only for small n + n_u (a few thousand): it costs O((n + n_u)^3).
"""
import numpy as np
import scipy.linalg as sla

from .covariance import k_cross, k_same


class Dense:
    """All dense matrices of one problem, indexed over V = [D ; U]."""

    def __init__(self, p):
        self.p = p
        n, M, B = p.n, p.M, int(p.B)
        self.n, self.M = n, M
        self.B = min(B, M - 1)
        U = p.U if p.U is not None else np.zeros((0, p.d))
        self.n_u = U.shape[0]
        P = np.vstack([p.X, U])
        # Sigma_VV with noise on the diagonal of V (D and U are each "same set").
        self.Sig = k_same(P, p.log_hyp)
        self.Sig_SS = k_same(p.S, p.log_hyp)
        self.K_VS = k_cross(P, p.S, p.log_hyp)
        self.Q = self.K_VS @ np.linalg.solve(self.Sig_SS, self.K_VS.T)
        self.R = self.Sig - self.Q
        bp = np.asarray(p.block_ptr)
        ubp = np.asarray(p.u_block_ptr) if p.U is not None else np.zeros(M + 1, dtype=np.int64)
        self.Didx = [np.arange(bp[m], bp[m + 1]) for m in range(M)]
        self.Uidx = [n + np.arange(ubp[m], ubp[m + 1]) for m in range(M)]
        self.Vidx = [np.r_[self.Didx[m], self.Uidx[m]] for m in range(M)]
        self.Rbar = self._rbar()
        self.Sbar = self.Q + self.Rbar
        self.c = p.y - p.prior_mean

    def DB(self, m):
        """D^B_m: the training inputs of the next B blocks (truncated at M)."""
        ks = range(m + 1, min(m + self.B, self.M - 1) + 1)
        if len(ks) == 0:
            return np.zeros(0, dtype=np.int64)
        return np.concatenate([self.Didx[k] for k in ks])

    def _rbar(self):
        """R_bar_VV block by block, Eq. (1).

        Blocks inside the B-band equal R.  Outside it (B > 0) the upper block
        (m, n), n - m > B, is R_{V_m D^B_m} R_{D^B_m D^B_m}^-1 R_bar_{D^B_m V_n}
        and the lower block (a, b), a - b > B, is
        R_bar_{V_a D^B_b} R_{D^B_b D^B_b}^-1 R_{D^B_b V_b}; both only use blocks
        closer to the diagonal, so they are filled in order of increasing
        distance from it.  With B = 0 the off-band blocks are zero.
        """
        M, B, R, V = self.M, self.B, self.R, self.Vidx
        N = R.shape[0]
        Rb = np.zeros((N, N))
        for m in range(M):
            for k in range(M):
                if abs(m - k) <= B:
                    Rb[np.ix_(V[m], V[k])] = R[np.ix_(V[m], V[k])]
        if B == 0:
            return Rb
        for dist in range(B + 1, M):
            for m in range(0, M - dist):
                k = m + dist
                Dm = self.DB(m)
                Rdd = R[np.ix_(Dm, Dm)]
                # upper block (m, k): case n - m > B > 0
                right = Rb[np.ix_(Dm, V[k])]
                Rb[np.ix_(V[m], V[k])] = R[np.ix_(V[m], Dm)] @ np.linalg.solve(Rdd, right)
                # lower block (k, m): case m - n > B > 0 with rows k, columns m
                left = Rb[np.ix_(V[k], Dm)]
                Rb[np.ix_(V[k], V[m])] = left @ np.linalg.solve(Rdd, R[np.ix_(Dm, V[m])])
        return Rb

    # views ---------------------------------------------------------------
    def block(self, A, rows, cols):
        return A[np.ix_(rows, cols)]

    @property
    def D(self):
        return np.arange(self.n)

    @property
    def Uall(self):
        return self.n + np.arange(self.n_u)

    def predict(self, full_cov=False):
        """Eqs. (3) and (4)."""
        D, U = self.D, self.Uall
        Sdd = self.Sbar[np.ix_(D, D)]
        Sud = self.Sbar[np.ix_(U, D)]
        F = sla.cho_factor(Sdd, lower=True)
        mean = self.p.prior_mean + Sud @ sla.cho_solve(F, self.c)
        cov = self.Sbar[np.ix_(U, U)] - Sud @ sla.cho_solve(F, Sud.T)
        return mean, (cov if full_cov else np.diag(cov).copy())

    def lml(self):
        """log N(y; mu 1, Sigma_bar_DD)."""
        D = self.D
        Sdd = self.Sbar[np.ix_(D, D)]
        L = np.linalg.cholesky(Sdd)
        a = sla.solve_triangular(L, self.c, lower=True)
        return float(-0.5 * a @ a - np.sum(np.log(np.diag(L))) - 0.5 * self.n * np.log(2 * np.pi))


def predict(p, full_cov=False):
    return Dense(p).predict(full_cov=full_cov)


def lml(p):
    return Dense(p).lml()


def lml_grad_fd(p, h=1e-5):
    """Central finite differences of the dense LML in log-hyperparameters."""
    g = np.zeros(p.d + 2)
    for j in range(p.d + 2):
        e = np.zeros(p.d + 2)
        e[j] = h
        g[j] = (lml(p.with_(log_hyp=p.log_hyp + e)) - lml(p.with_(log_hyp=p.log_hyp - e))) / (2 * h)
    return g
