"""Squared-exponential ARD covariance (Section "Experiments", covariance
function with signal variance, noise variance and one length-scale per input
dimension).  Oracle: test infrastructure only.

Hyperparameter vector theta (log scale): [log l_1 .. log l_d, log sigma_s^2,
log sigma_n^2].  Noise follows the index reading: it is added only on the
diagonal of a set with itself.
"""
import numpy as np
from scipy.spatial.distance import cdist


def unpack(log_hyp, d):
    log_hyp = np.asarray(log_hyp, dtype=np.float64)
    assert log_hyp.shape == (d + 2,)
    return np.exp(log_hyp[:d]), float(np.exp(log_hyp[d])), float(np.exp(log_hyp[d + 1]))


def k_cross(A, B, log_hyp):
    """sigma_s^2 exp(-0.5 sum_i (a_i - b_i)^2 / l_i^2); no noise term."""
    d = A.shape[1]
    ell, sf2, _ = unpack(log_hyp, d)
    if A.shape[0] == 0 or B.shape[0] == 0:
        return np.zeros((A.shape[0], B.shape[0]))
    d2 = cdist(A / ell, B / ell, "sqeuclidean")
    return sf2 * np.exp(-0.5 * d2)


def k_same(A, log_hyp):
    """Covariance of a set with itself: k_cross(A, A) + sigma_n^2 I."""
    d = A.shape[1]
    _, _, sn2 = unpack(log_hyp, d)
    K = k_cross(A, A, log_hyp)
    K[np.diag_indices_from(K)] += sn2
    return K


def dk_cross(A, B, log_hyp):
    """Derivatives of k_cross(A, B) with respect to each entry of theta.

    d/d log l_i     = k * (a_i - b_i)^2 / l_i^2
    d/d log sigma_s^2 = k
    d/d log sigma_n^2 = 0 (cross-set blocks carry no noise)
    """
    d = A.shape[1]
    ell, _, _ = unpack(log_hyp, d)
    K = k_cross(A, B, log_hyp)
    out = []
    for i in range(d):
        diff = (A[:, i][:, None] - B[:, i][None, :]) / ell[i]
        out.append(K * diff * diff)
    out.append(K.copy())
    out.append(np.zeros_like(K))
    return out


def dk_same(A, log_hyp):
    """Derivatives of k_same(A) with respect to theta; the noise entry is
    sigma_n^2 I."""
    d = A.shape[1]
    _, _, sn2 = unpack(log_hyp, d)
    out = dk_cross(A, A, log_hyp)
    out[d + 1] = sn2 * np.eye(A.shape[0])
    return out
