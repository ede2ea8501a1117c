"""Scalable LMA in whitened-window form (oracle tier O2).  Test
infrastructure only.

Notation (blocks 0..M-1 in the given Markov order):
  W_m = D^B_m, the training inputs of blocks m+1 .. min(m+B, M-1);
  J_m = [W_m ; D_m] in that order; c = y - mu.
  V_X = L_SS^-1 K_SX with L_SS = chol(Sigma_SS), so Q_XX' = V_X^T V_X'.
  R_X = Sigma_XX - V_X^T V_X (noise on the diagonal of same-set blocks).

Window factorisation (Lemma 1 with Definition 1).  With L_m = chol(R_{J_m}) =
[[L11, 0], [L21, L22]]:  R'_m = L21 L11^-1, Rdot_m^-1 = L22 L22^T, hence the
last |D_m| rows of L_m^-1 [K_{J S} | c_J] are Z_m = L22^-1 Sdot^m_S and
z_m = L22^-1 ydot_m, so Sdot^T Rdot Sdot = Z^T Z and Sdot^T Rdot ydot = Z^T z.

Global summary (Definition 2):  Sigma_ddot_SS = Sigma_SS + sum Z_m^T Z_m,
y_ddot_S = sum Z_m^T z_m, g = Sigma_ddot_SS^-1 y_ddot_S.

Log marginal likelihood via Eq. (5) and the determinant lemma:
  log|Sigma_bar_DD| = sum_m log|Rdot_m^-1| + log|Sigma_ddot_SS| - log|Sigma_SS|
  c^T Sigma_bar^-1 c = sum_m |z_m|^2 - y_ddot_S^T g.

Prediction for u in test block q (Theorem 2 restricted to the windows whose
rows of the banded Cholesky factor of R_bar_DD^-1 touch u):
  x^m_u = last |D_m| rows of L_m^-1 R_{J_m u}   for m = max(0, q-B) .. q,
  pi_u  = L11(q)^-1 R_{W_q u},
  G_u = sum_m Z_m^T x^m_u + Pi_q^T pi_u,   l_u = sum_m z_m^T x^m_u + p_q^T pi_u,
  xi_u = sum_m |x^m_u|^2 + |pi_u|^2,
  mean_u = mu + (k_u - G_u)^T g + l_u,
  var_u  = sigma_s^2 + sigma_n^2 - |L_SS^-1 k_u|^2 - xi_u
           + (k_u - G_u)^T Sigma_ddot_SS^-1 (k_u - G_u),
where k_u = K_{S u}, Pi_q and p_q are the first |W_q| rows of L_q^-1 [K_JS | c_J].
Windows below q-B contribute nothing beyond the low-rank part (their rows of the
factor map R_bar_{D u} to zero by the recursion of Eq. (1)), and those above q
collapse onto the single W_q term.

All in one pass over windows: window m's triangular solve carries the test
right-hand sides of blocks q = m .. m+B, and the per-point sums finish once g is
known.

Full predictive covariance (Eq. (4) beyond its diagonal; predict_cov).  With
E_u = k_u - G_u, Eq. (4) through the matrix inversion lemma of Eq. (5) is
  Sigma_uv = R_bar_uv - xi_uv + E_u^T Sigma_ddot_SS^-1 E_v,
  xi_uv = R_bar_uD R_bar_DD^-1 R_bar_Dv.
For u in test block q and v in block r with |q - r| <= B, R_bar_uv = R_uv
(Eq. (1) inside the band; noise on the diagonal) and, with a = min(q, r),
b = max(q, r),
  xi_uv = sum_{m=b-B}^{a-1} x^m_u . x^m_v  +  X^a_u . X^a_v,
where X^a_u is the whole column of L_a^-1 R_{J_a u} (its first |W_a| rows are
pi_u when a = q): the windows below b-B hold no whitened part of v, and the
windows above a collapse onto W_a as for the diagonal.  For |q - r| > B, Eq. (1)
gives R_bar_uv = pi_u . L11(q)^-1 R_bar_{W_q v} (q < r), which is also all of
xi_uv, so the two cancel and only the low-rank term E_u^T Sigma_ddot^-1 E_v is
left: given the training outputs, test points more than B blocks apart are
uncorrelated in the residual.  (Pinned against the dense definition.)
"""
import numpy as np
import scipy.linalg as sla

from .covariance import k_cross, k_same, unpack, dk_cross, dk_same

LOG2PI = float(np.log(2.0 * np.pi))


def window_index(block_ptr, M, B, m):
    """(W_m indices, D_m indices) into the rows of X."""
    bp = block_ptr
    hi = min(m + B, M - 1)
    W = np.arange(bp[m + 1], bp[hi + 1]) if hi > m else np.zeros(0, dtype=np.int64)
    Dm = np.arange(bp[m], bp[m + 1])
    return W, Dm


class Fit:
    """Fit state: L_SS, V = L_SS^-1 K_SD, the global summary and its solve."""

    def __init__(self, p, windows=None, test=True, keep_test_cols=False):
        self.p = p
        self.keep = keep_test_cols
        self.Xcols = {}
        n, d, M = p.n, p.d, p.M
        self.B = min(int(p.B), M - 1)
        self.ell, self.sf2, self.sn2 = unpack(p.log_hyp, d)
        self.c = p.y - p.prior_mean
        self.Sig_SS = k_same(p.S, p.log_hyp)
        self.L_SS = np.linalg.cholesky(self.Sig_SS)
        self.K_SD = k_cross(p.S, p.X, p.log_hyp)
        self.V = sla.solve_triangular(self.L_SS, self.K_SD, lower=True)
        s = p.s
        self.test = test and p.U is not None and p.U.shape[0] > 0
        if self.test:
            self.K_SU = k_cross(p.S, p.U, p.log_hyp)
            self.V_U = sla.solve_triangular(self.L_SS, self.K_SU, lower=True)
            n_u = p.U.shape[0]
            self.G = np.zeros((n_u, s))
            self.l_u = np.zeros(n_u)
            self.xi = np.zeros(n_u)
        self.Sdd_acc = np.zeros((s, s))
        self.ydd = np.zeros(s)
        self.qsum = 0.0
        self.ldR = 0.0
        for m in (range(M) if windows is None else windows):
            self.window(m)

    def R_block(self, A, B_, same):
        """Residual covariance R between two index sets of D (or D and U)."""
        p = self.p
        if same:
            K = k_same(p.X[A], p.log_hyp)
        else:
            K = k_cross(p.X[A], p.X[B_], p.log_hyp)
        return K - self.V[:, A].T @ self.V[:, B_]

    def window(self, m):
        p, B, M, s = self.p, self.B, self.p.M, self.p.s
        W, Dm = window_index(p.block_ptr, M, B, m)
        J = np.r_[W, Dm]
        w = W.size
        RJ = k_same(p.X[J], p.log_hyp) - self.V[:, J].T @ self.V[:, J]
        L = np.linalg.cholesky(RJ)
        cols = [self.K_SD[:, J].T, self.c[J][:, None]]
        qs = []
        if self.test:
            ubp = p.u_block_ptr
            for q in range(m, min(m + B, M - 1) + 1):
                uq = np.arange(ubp[q], ubp[q + 1])
                if uq.size == 0:
                    continue
                RJu = k_cross(p.X[J], p.U[uq], p.log_hyp) - self.V[:, J].T @ self.V_U[:, uq]
                qs.append((q, uq, sum(c.shape[1] for c in cols)))
                cols.append(RJu)
        sol = sla.solve_triangular(L, np.hstack(cols), lower=True)
        Z, z = sol[w:, :s], sol[w:, s]
        self.Sdd_acc += Z.T @ Z
        self.ydd += Z.T @ z
        self.qsum += float(z @ z)
        self.ldR += 2.0 * float(np.sum(np.log(np.diag(L)[w:])))
        for q, uq, off in qs:
            X_ = sol[:, off:off + uq.size]
            if self.keep:
                self.Xcols[(m, q)] = (X_.copy(), w)
            x = X_[w:]
            self.G[uq] += x.T @ Z
            self.l_u[uq] += x.T @ z
            self.xi[uq] += np.sum(x * x, axis=0)
            if q == m and w > 0:
                pi = X_[:w]
                self.G[uq] += pi.T @ sol[:w, :s]
                self.l_u[uq] += pi.T @ sol[:w, s]
                self.xi[uq] += np.sum(pi * pi, axis=0)

    def finish(self):
        self.Sdd = self.Sig_SS + self.Sdd_acc
        self.L_dd = np.linalg.cholesky(self.Sdd)
        self.g = sla.cho_solve((self.L_dd, True), self.ydd)
        return self

    def lml(self):
        n = self.p.n
        ld_dd = 2.0 * np.sum(np.log(np.diag(self.L_dd)))
        ld_ss = 2.0 * np.sum(np.log(np.diag(self.L_SS)))
        quad = self.qsum - float(self.ydd @ self.g)
        return float(-0.5 * (quad + self.ldR + ld_dd - ld_ss + n * LOG2PI))

    def predict(self):
        E = self.K_SU.T - self.G
        mean = self.p.prior_mean + E @ self.g + self.l_u
        T = sla.solve_triangular(self.L_dd, E.T, lower=True)
        var = (self.sf2 + self.sn2 - np.sum(self.V_U ** 2, axis=0) - self.xi
               + np.sum(T * T, axis=0))
        return mean, var


    def predict_cov(self):
        """Full predictive covariance over the test points (needs a fit made
        with keep_test_cols=True)."""
        p, B, M = self.p, self.B, self.p.M
        ubp = p.u_block_ptr
        n_u = p.U.shape[0]
        E = self.K_SU.T - self.G
        T = sla.solve_triangular(self.L_dd, E.T, lower=True)
        cov = T.T @ T
        for q in range(M):
            uq = np.arange(ubp[q], ubp[q + 1])
            for r in range(q, min(q + B, M - 1) + 1):
                vr = np.arange(ubp[r], ubp[r + 1])
                if uq.size == 0 or vr.size == 0:
                    continue
                Rqr = k_cross(p.U[uq], p.U[vr], p.log_hyp) - self.V_U[:, uq].T @ self.V_U[:, vr]
                if q == r:
                    Rqr[np.diag_indices_from(Rqr)] += self.sn2
                xi = np.zeros((uq.size, vr.size))
                for m in range(max(0, r - B), q):          # D rows of the windows below q
                    Xu, w = self.Xcols[(m, q)]
                    Xv, _ = self.Xcols[(m, r)]
                    xi += Xu[w:].T @ Xv[w:]
                Xu, _ = self.Xcols[(q, q)]                   # all rows of window q
                Xv, _ = self.Xcols[(q, r)]
                xi += Xu.T @ Xv
                cov[np.ix_(uq, vr)] += Rqr - xi
                if r != q:
                    cov[np.ix_(vr, uq)] += (Rqr - xi).T
        return cov


def predict_cov(p):
    """Predictive mean and full covariance at the test inputs."""
    f = Fit(p, keep_test_cols=True).finish()
    mean, _ = f.predict()
    return mean, f.predict_cov()


def fit_predict(p):
    """Predictive mean and variance (diagonal) at the test inputs, plus the
    log marginal likelihood, in one pass over the windows."""
    f = Fit(p).finish()
    mean, var = f.predict()
    return dict(mean=mean, var=var, lml=f.lml(), g=f.g, Sdd=f.Sdd, ydd=f.ydd)


def lml(p):
    return Fit(p, test=False).finish().lml()


# --------------------------------------------------------------------------
# adjoint of the log marginal likelihood
# --------------------------------------------------------------------------

def lml_grad(p):
    """LML and its gradient in theta = [log l, log sigma_s^2, log sigma_n^2].

    R_bar_DD^-1 is a signed sum over windows X of zero-padded R_X^-1, with
    sign +1 for J_m and -1 for W_m (from the block rows of its banded Cholesky
    factor), and log|R_bar_DD| = sum sign * log|R_X|.  Differentiating
      LML = -1/2 [ sum_X sign (c_X^T R_X^-1 c_X + log|R_X|) - y_ddot^T Sigma_ddot^-1 y_ddot
                   + log|Sigma_ddot| - log|Sigma_SS| + n log 2 pi ]
    with R_X = Sigma_XX - K_XS Sigma_SS^-1 K_SX gives, with alpha = R_X^-1 c_X,
    Gamma = R_X^-1 K_XS, g = Sigma_ddot^-1 y_ddot, H = Sigma_ddot^-1, beta = Gamma g:
      Rb_X  = sign/2 [ (alpha-beta)(alpha-beta)^T - R_X^-1 + Gamma H Gamma^T ]
      Kb_SX = sign [ g (alpha-beta)^T - H Gamma^T ] - 2 Sigma_SS^-1 K_SX Rb_X
      Sb_SS = 1/2 Sigma_SS^-1 - 1/2 (g g^T + H)
              + sum_X Sigma_SS^-1 K_SX Rb_X K_XS Sigma_SS^-1
      dLML/dtheta_j = sum_X <Rb_X, dSigma_XX/dtheta_j> + <Kb_SX, dK_SX/dtheta_j>
                      + <Sb_SS, dSigma_SS/dtheta_j>.
    """
    f = Fit(p, test=False).finish()
    lml_val = f.lml()
    d, M, B = p.d, p.M, f.B
    H = sla.cho_solve((f.L_dd, True), np.eye(p.s))
    g = f.g
    Sig_SS_inv = sla.cho_solve((f.L_SS, True), np.eye(p.s))
    grad = np.zeros(d + 2)
    Sb = 0.5 * Sig_SS_inv - 0.5 * (np.outer(g, g) + H)
    for m in range(M):
        W, Dm = window_index(p.block_ptr, M, B, m)
        J = np.r_[W, Dm]
        for X, sign in ((J, 1.0), (W, -1.0)):
            if X.size == 0:
                continue
            RX = k_same(p.X[X], p.log_hyp) - f.V[:, X].T @ f.V[:, X]
            LX = np.linalg.cholesky(RX)
            RXi = sla.cho_solve((LX, True), np.eye(X.size))
            K_XS = f.K_SD[:, X].T
            alpha = RXi @ f.c[X]
            Gam = RXi @ K_XS
            beta = Gam @ g
            ab = alpha - beta
            Rb = 0.5 * sign * (np.outer(ab, ab) - RXi + Gam @ H @ Gam.T)
            A = Sig_SS_inv @ K_XS.T  # Sigma_SS^-1 K_SX
            Kb = sign * (np.outer(g, ab) - H @ Gam.T) - 2.0 * A @ Rb
            Sb += A @ Rb @ A.T
            dS = dk_same(p.X[X], p.log_hyp)
            dK = dk_cross(p.S, p.X[X], p.log_hyp)
            for j in range(d + 2):
                grad[j] += np.sum(Rb * dS[j]) + np.sum(Kb * dK[j])
    dSS = dk_same(p.S, p.log_hyp)
    for j in range(d + 2):
        grad[j] += np.sum(Sb * dSS[j])
    return lml_val, grad
