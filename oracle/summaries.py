"""The paper's own route to the LMA prediction (oracle tier O1).  Test
infrastructure only.

Local summary (Definition 1), for block m with D^B_m the next B blocks:
  R'_m      = R_{D_m D^B_m} R_{D^B_m D^B_m}^-1
  ydot_m    = (y - mu)_{D_m} - R'_m (y - mu)_{D^B_m}
  Rdot_m    = (R_{D_m D_m} - R'_m R_{D^B_m D_m})^-1
  Sdot^m_S  = Sigma_{D_m S} - R'_m Sigma_{D^B_m S}
  Sdot^m_U  = Sigma_bar_{D_m U} - R'_m Sigma_bar_{D^B_m U}
Global summary (Definition 2): sums over m of Sdot^T Rdot ydot, Sdot^T Rdot Sdot,
with Sigma_ddot_SS = Sigma_SS + sum_m Sdot^m_S^T Rdot_m Sdot^m_S.
Prediction (Theorem 2):
  mean = mu + y_ddot_U - Sigma_ddot_US Sigma_ddot_SS^-1 y_ddot_S
  cov  = Sigma_UU - Sigma_ddot_UU + Sigma_ddot_US Sigma_ddot_SS^-1 Sigma_ddot_US^T
Sigma_bar_{D U} is taken from the dense tier; with an empty D^B_m (last block,
or B = 0) the terms with R'_m vanish.
"""
import numpy as np

from .dense import Dense


def local_summary(dn: Dense, m: int):
    R = dn.R
    Dm, DB = dn.Didx[m], dn.DB(m)
    c = dn.c
    U = dn.Uall
    Sig_DS = dn.K_VS  # cross covariance with S has no noise term
    if DB.size:
        Rp = R[np.ix_(Dm, DB)] @ np.linalg.inv(R[np.ix_(DB, DB)])
    else:
        Rp = np.zeros((Dm.size, 0))
    ydot = c[Dm] - Rp @ c[DB]
    Rdot = np.linalg.inv(R[np.ix_(Dm, Dm)] - Rp @ R[np.ix_(DB, Dm)])
    SdS = Sig_DS[Dm] - Rp @ Sig_DS[DB]
    SdU = dn.Sbar[np.ix_(Dm, U)] - Rp @ dn.Sbar[np.ix_(DB, U)]
    return dict(Rp=Rp, ydot=ydot, Rdot=Rdot, SdS=SdS, SdU=SdU)


def global_summary(dn: Dense):
    s, n_u = dn.Sig_SS.shape[0], dn.n_u
    yS, yU = np.zeros(s), np.zeros(n_u)
    SSS, SUS, SUU = dn.Sig_SS.copy(), np.zeros((n_u, s)), np.zeros((n_u, n_u))
    for m in range(dn.M):
        ls = local_summary(dn, m)
        Rd = ls["Rdot"]
        yS += ls["SdS"].T @ Rd @ ls["ydot"]
        yU += ls["SdU"].T @ Rd @ ls["ydot"]
        SSS += ls["SdS"].T @ Rd @ ls["SdS"]
        SUS += ls["SdU"].T @ Rd @ ls["SdS"]
        SUU += ls["SdU"].T @ Rd @ ls["SdU"]
    return dict(yS=yS, yU=yU, SSS=SSS, SUS=SUS, SUU=SUU)


def predict(p, full_cov=False):
    dn = Dense(p)
    gs = global_summary(dn)
    U = dn.Uall
    mean = p.prior_mean + gs["yU"] - gs["SUS"] @ np.linalg.solve(gs["SSS"], gs["yS"])
    cov = dn.Sig[np.ix_(U, U)] - gs["SUU"] + gs["SUS"] @ np.linalg.solve(gs["SSS"], gs["SUS"].T)
    return mean, (cov if full_cov else np.diag(cov).copy())
