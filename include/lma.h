/*
 * lma.h -- C ABI of the MI355X (gfx950) library for the low-rank-cum-Markov
 * approximation (LMA) of Gaussian-process regression.
 *
 * Low, Yu, Chen, Jaillet, "Parallel Gaussian Process Regression for Big Data:
 * Low-Rank Representation Meets Markov Approximation", AAAI 2015.
 *
 * Conventions for every entry point
 *   - Array pointers are DEVICE pointers unless marked (host).  Matrices are
 *     row-major.  The caller owns every buffer passed in; the library never
 *     frees caller memory and writes outputs only into caller buffers.
 *   - Work is ordered on the given HIP stream (0 = the null stream).  lma_fit
 *     and lma_lml synchronise that stream once at the end to read the status
 *     word; lma_predict synchronises once too.
 *   - Errors are returned as a status code; nothing is silently regularised.
 *     lma_last_error() gives a message for the calling thread and
 *     lma_failed_block() the block whose residual covariance was not positive
 *     definite.
 *   - A state is not reentrant: do not use one lma_state from two threads or
 *     two streams at once.
 */
#ifndef LMA_H
#define LMA_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LMA_OK = 0,
  LMA_E_ARG = 1,     /* invalid argument (shape, pointer, partition) */
  LMA_E_NOT_PD = 2,  /* a covariance that must be positive definite is not */
  LMA_E_HIP = 3,     /* HIP runtime error */
  LMA_E_NOMEM = 4,   /* device memory for the state could not be allocated */
  LMA_E_INTERNAL = 5 /* any other failure inside the library (message in
                        lma_last_error); no exception ever leaves an entry point */
} lma_status;

typedef enum {
  LMA_FP64 = 0,   /* every step in float64 */
  LMA_MIXED = 1   /* window assembly, Cholesky and solves in float32 on MFMA;
                     Sigma_SS, V = L_SS^-1 K_SD, the summary reduction, the
                     global |S|x|S| system and the prediction combine in float64 */
} lma_precision;

/*
 * The regression problem, following the problem statement of the paper:
 *   D with outputs y, partitioned into M blocks D_1..D_M (Section
 *   "Low-Rank-cum-Markov Approximation": the partition of D and U);
 *   support set S (reduced-rank representation over S);
 *   Markov order B in {0..M-1} (Eq. (1); B = 0 is PIC, B = M-1 the full GP);
 *   squared-exponential ARD covariance with hyperparameters
 *   sigma_s^2, sigma_n^2, l_1..l_d (Section "Experiments") and a constant
 *   prior mean.
 * Noise sigma_n^2 is added on the diagonal of same-set blocks (D with D,
 * U with U, S with S) only, never on cross-set blocks.
 */
typedef struct {
  int64_t n;                  /* |D| >= 1 */
  int64_t d;                  /* input dimension, 1..64 */
  int64_t s;                  /* |S| >= 1 */
  int64_t M;                  /* number of blocks >= 1 */
  int64_t B;                  /* Markov order >= 0; values >= M-1 are clamped to M-1 */
  const double *X;            /* [n,d]; block m = rows block_ptr[m] .. block_ptr[m+1]-1,
                                 blocks in Markov order (D^B_m = the next B blocks) */
  const double *y;            /* [n] outputs */
  const int64_t *block_ptr;   /* (host) [M+1], 0 = p[0] < p[1] < ... < p[M] = n */
  const double *S;            /* [s,d] support inputs */
  const double *log_hyp;      /* (host) [d+2] = log l_1..log l_d, log sigma_s^2, log sigma_n^2 */
  double prior_mean;          /* constant prior mean mu */
  int32_t precision;          /* lma_precision */
  int32_t reserved;           /* must be 0 */
  int64_t mem_budget_bytes;   /* 0 = no limit.  Otherwise the state stays within it: when every
                                 window's factor does not fit, the windows are processed in chunks
                                 and refactored by each pass that needs them (lma_state_chunks);
                                 LMA_E_NOMEM when not even one window fits */
} lma_problem;

/* Opaque fit state, owned by the library (release with lma_free).  Holds the
 * Cholesky factor of Sigma_SS, the factors of every window residual
 * covariance R_{J_m} (J_m = [D^B_m ; D_m]), the whitened support rows of each
 * window, the Cholesky factor of the global matrix Sigma_ddot_SS and
 * g = Sigma_ddot_SS^-1 y_ddot_S (Definition 2, Theorem 2). */
typedef struct lma_state lma_state;

/*
 * Fit: local summaries of every block (Definition 1, computed through the
 * banded Cholesky factor of Lemma 1), their reduction into the global summary
 * (Definition 2) and the factorisation of Sigma_ddot_SS.  The problem's
 * arrays are copied/consumed during the call; the caller may free them
 * afterwards.  On success *out receives a new state; on failure *out is NULL.
 * Errors: LMA_E_ARG, LMA_E_NOT_PD (lma_failed_block: m for the window of block
 * m, -1 for Sigma_SS, -2 for Sigma_ddot_SS), LMA_E_HIP, LMA_E_NOMEM.
 */
lma_status lma_fit(const lma_problem *p, hipStream_t stream, lma_state **out);

/*
 * Predict (Theorem 2; Eqs. (3)-(4)) at n_u test inputs U partitioned into the
 * same M blocks: test block q = rows u_block_ptr[q] .. u_block_ptr[q+1]-1
 * (empty blocks allowed).  mean[i] is the predictive mean, var[i] (if var is
 * not NULL) the predictive variance of the noisy output (diagonal of
 * Sigma^LMA_UU), returned as Eq. (4) defines it, without clamping: it never
 * exceeds sigma_s^2 + sigma_n^2, and for 0 < B < M-1 it can be negative at a
 * few test points, because the covariance of Eq. (2) over training and test
 * inputs together need not be positive definite there.
 * Errors: LMA_E_ARG, LMA_E_HIP, LMA_E_NOMEM.
 */
lma_status lma_predict(lma_state *f, int64_t n_u, const double *U, const int64_t *u_block_ptr,
                       double *mean, double *var, hipStream_t stream);

/*
 * Full predictive covariance (Theorem 2's Sigma^LMA_UU, Eq. (4) beyond its
 * diagonal) at n_u test inputs partitioned as for lma_predict.  cov [n_u][n_u]
 * (row-major, caller-owned, n_u^2 doubles) receives the covariance of the
 * noisy test outputs, computed as
 *   cov_uv = [|q - r| <= B] (R_uv - xi_uv) + E_u^T Sigma_ddot_SS^-1 E_v
 * for u in test block q and v in test block r: R the residual covariance
 * (noise on the diagonal), xi_uv the product of the two points' whitened
 * window rows over the windows that hold both, E_u = K_Su - G_u as for the
 * variance.  For test blocks more than B apart the residual part of Eq. (1)
 * cancels exactly, so their entries are the low-rank term alone.  Its
 * diagonal is lma_predict's variance; it is symmetric up to rounding and, for
 * 0 < B < M-1, need not be positive semidefinite.  mean [n_u] (or NULL)
 * receives the predictive mean.  Meant for small test sets: the work and the
 * output grow as n_u^2.  Synchronises the stream.
 * Errors: LMA_E_ARG (also n_u > 2^31), LMA_E_HIP, LMA_E_NOMEM.
 */
lma_status lma_predict_cov(lma_state *f, int64_t n_u, const double *U, const int64_t *u_block_ptr,
                           double *mean, double *cov, hipStream_t stream);

/*
 * Log marginal likelihood log N(y; mu, Sigma_bar_DD) of the LMA prior
 * (through the matrix inversion lemma of Eq. (5) and the block factor of
 * Lemma 1), written to *lml (host).  If grad (host, [d+2]) is not NULL it
 * receives the gradient with respect to log_hyp = (log l_1..log l_d,
 * log sigma_s^2, log sigma_n^2), from the reverse-mode adjoint of the same
 * computation (the prior mean is held fixed).  The gradient pass processes
 * the windows in chunks whose workspace stays under the part of
 * mem_budget_bytes the fitted state leaves (at least 256 MB; 16 GB when
 * mem_budget_bytes is 0).  Synchronises the stream.  Errors as for lma_fit;
 * LMA_E_NOT_PD also for a non-finite gradient.
 */
lma_status lma_lml(const lma_problem *p, double *lml, double *grad, hipStream_t stream);

/* Release a state (NULL is ignored).  Its device memory is kept for reuse by
 * the next lma_fit / lma_predict of a similar size (at most four blocks are
 * kept per process); lma_release_cache() hands them back to the runtime. */
void lma_free(lma_state *f);

/* Free the device blocks kept for reuse. */
void lma_release_cache(void);

/* LML of a fitted state (host scalar) without recomputation. */
lma_status lma_state_lml(const lma_state *f, double *lml);

/* Device bytes a fitted state holds, and the number of chunks its window
 * factors are processed in: 1 when every window's factor is resident; more
 * when mem_budget_bytes was too small for that, in which case the state holds
 * one chunk of windows at a time and lma_predict / lma_lml refactor the
 * windows chunk by chunk (same arithmetic as the fit).  Both return -1 for a
 * NULL state. */
int64_t lma_state_bytes(const lma_state *f);
int64_t lma_state_chunks(const lma_state *f);

/* Message for the last error on the calling thread ("" if none). */
const char *lma_last_error(void);

/* Which factor the last lma_fit / lma_predict / lma_lml on the calling thread
 * failed on with LMA_E_NOT_PD: m (0..M-1) for the window of block m, -1 for
 * Sigma_SS, -2 for Sigma_ddot_SS.  -3 when that call did not fail on a factor:
 * it succeeded, failed with another status, or found a non-finite log
 * marginal likelihood or gradient, which no single block is blamed for.
 * Every one of those entry points resets it to -3 when it starts. */
int64_t lma_failed_block(void);

/*
 * Live kernel timing (for benchmarks).  When enabled, every launch of the
 * engine's kernels is bracketed by HIP events on the caller's stream; the
 * elapsed times are summed at the end of each lma_fit / lma_predict call
 * (which synchronise anyway).  update_alg_flops counts the multiply-adds of
 * the update launches on real entries only (no tile padding), 2 flops each:
 * the Cholesky updates, the Q = V^T V correction of the residual and the
 * right-hand-side updates.  Tile GEMMs and gradient contractions are timed in
 * their own fields (not in other_ms).  Not thread safe; for single-threaded use.
 */
typedef struct {
  double update_ms;          /* summed device time of update launches */
  double diag_ms;            /* diagonal-tile factor + inverse launches */
  double trsm_ms;            /* off-diagonal triangular-solve launches */
  double other_ms;           /* every other kernel of the library */
  double update_alg_flops;   /* algorithmic flops of the timed update launches */
  double update_alg_flops_f64; /* the part of them done on float64 matrix cores */
  int64_t update_launches;
  int64_t other_launches;    /* launches counted in other_ms */
  double gemm_ms;            /* batched tile GEMMs (summaries, prediction sums, gradient products) */
  double gemm_alg_flops;     /* 2 x multiply-adds on their valid output entries */
  double contract_ms;        /* gradient contractions (adjoint tile x covariance derivatives) */
  double contract_alg_flops; /* 2 x multiply-adds of their tile products on valid entries */
  int64_t gemm_launches;
  int64_t contract_launches;
} lma_profile;

void lma_profile_enable(int on);
/* Copy the accumulated figures into *out; reset them if reset != 0. */
lma_status lma_profile_read(lma_profile *out, int reset);

/* Library version string. */
const char *lma_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LMA_H */
