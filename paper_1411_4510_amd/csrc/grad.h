// Kernels of the log-marginal-likelihood adjoint (grad.hip).
//
// Every term of the gradient has the form <A, dK/dtheta> with A an adjoint
// matrix (of a residual window, of K_SX or of Sigma_SS) and K the SE-ARD
// covariance of two point sets.  A contraction item computes one 128 x 128
// tile of A as a signed sum of tile GEMMs, rank-one terms and explicit
// matrices, regenerates the covariance tile from the scaled coordinates and
// reduces
//   sum_ij A_ij k_ij (dx_ij,q)^2   (q < d: d/d log l_q),
//   sum_ij A_ij k_ij               (d/d log sigma_s^2),
//   sum_i  A_ii sigma_n^2          (d/d log sigma_n^2, same-set diagonal tiles)
// to d+2 numbers; a fixed-order reduction over the items gives the gradient.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.h"

namespace lma {

enum DcKind : int32_t { DC_SAME = 0, DC_CROSS = 1 };

struct DcItem {
  int32_t x0, x1;          // TX terms [x0, x1), all subtracted
  int32_t t0, tneg, t1;    // float64 terms: [t0, tneg) subtracted, [tneg, t1) added
  int32_t kind;            // DC_SAME: covariance of one point set (noise on the diagonal); DC_CROSS
  int32_t nr, nc;          // valid rows / columns of the tile
  int32_t diag;            // 1: tile on the diagonal of a same-set matrix
  int32_t nr1, nex;        // rank-one / explicit terms in use (at most 2 each)
  int32_t pad_;
  double wt;               // weight of the tile in the contraction
  const double* xr;        // scaled coordinates of the tile's rows [r][d]
  const double* xc;        // and columns [c][d]
  const double* r1a[2];    // rank-one terms r1s * r1a[row] * r1b[col]
  const double* r1b[2];
  double r1s[2];
  const double* ex[2];     // explicit terms exs * ex[row * exld + col]
  int64_t exld[2];
  double exs[2];
};

template <typename TX>
struct DcArgs {
  const DcItem* items;
  int32_t nitems;
  int32_t d;
  const GemmTerm<TX>* xterms;
  const GemmTerm<double>* terms;
  double sf2, sn2;
  double* partial;         // [item][d+2]
};

template <typename TX>
void launch_dcontract(const DcArgs<TX>& a, hipStream_t st);
// out[q] = sum over items i (fixed order) of partial[i * ncomp + q], q < ncomp
void launch_reduce_partials(const double* partial, int64_t nitems, int ncomp, double* out, hipStream_t st);
// Sigma_SS = K(S, S) + sigma_n^2 I as an sp x sp matrix, identity on the padding diagonal
void launch_sig_ss(const double* Ss, int s, int sp, int d, double sf2, double sn2, double* out, hipStream_t st);
// out = alpha * a + beta * b (n elements)
void launch_lincomb(double* out, const double* a, double alpha, const double* b, double beta, int64_t n,
                    hipStream_t st);
// u[x][t] = g[t] - hT[t * ldh + x] for x < nx, t < sp
void launch_uvec(double* u, const double* g, const double* hT, int64_t ldh, int nx, int sp, hipStream_t st);
// out[e] = a[e] - b[e] + sum_{k < ng} parts[k * n + e]  (fixed order)
void launch_sum_groups(double* out, const double* a, const double* b, const double* parts, int ng, int64_t n,
                       hipStream_t st);
hipError_t grad_init();

}  // namespace lma
