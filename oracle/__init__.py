"""CPU FP64 oracle for the low-rank-cum-Markov approximation (LMA) of GP regression.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library and its Python
binding never do.

Three tiers, all numpy/scipy in float64, sharing no code with the GPU path:

  dense      the definition: R_bar by the recursion of Eq. (1), Sigma_bar of
             Eq. (2), predictive mean/covariance of Eqs. (3)-(4), and the
             Gaussian log marginal likelihood under Sigma_bar_DD.
  summaries  the paper's own route: local summaries (Definition 1), global
             summary (Definition 2) and the prediction of Theorem 2.
  lma        the scalable form used at large n: whitened windows
             (Lemma 1 with Definition 1), the global summary, exact local
             prediction per test block, the log marginal likelihood through
             the matrix inversion lemma of Eq. (5), and its adjoint.

Beside them: deepsets (the warm-start network with the kernels' bfloat16
roundings) and kmeans (the partitioner's k-means steps and block chain order,
in the evaluation order the library fixes).

Readings of the paper the oracle takes (where it is silent):
  * noise is attached by index: sigma_n^2 sits on the diagonal of same-set
    blocks (D with D, U with U, S with S) and never on cross-set blocks, even
    where a support input coincides with a training input;
  * the predictive variance is that of the noisy output Y_u;
  * the prior mean is one constant mu;
  * D^B_m is the next B blocks, truncated at M; the block order is an input;
  * Theorem 2 is used for every B >= 0 (at B = 0 it reduces to PIC);
  * only the diagonal of the predictive covariance is returned, unclamped: it
    can be negative for 0 < B < M - 1, where Sigma_bar over D and U together
    is indefinite.
"""
from . import covariance, dense, summaries, lma  # noqa: F401
