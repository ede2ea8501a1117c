/*
 * lma_part.h -- C ABI of the clustering steps that partition the data into
 * blocks (gfx950).
 *
 * LMA needs the training and test inputs partitioned into M blocks, ordered
 * so that the B blocks after each one are its most correlated neighbours
 * (section "Low-Rank-cum-Markov Approximation"; the paper takes the
 * clustering from earlier work and does not specify it).  The library
 * takes the partition as an input (block_ptr in lma.h); these entry points
 * compute one on the GPU: k-means++ seeding, Lloyd's iteration (nearest-centre
 * assignment and centre update), a capacity-bounded assignment that keeps
 * every block between lo and hi points, the order of the blocks along the
 * Markov chain, and lma_partition, which composes them into block-contiguous
 * permutations of the training and test points.
 *
 * Arithmetic (fixed, so that results are reproducible bit for bit):
 *   - squared distance of point p to centre c: the sum over t = 0..d-1, in that
 *     order, of (p_t - c_t)^2, each difference, product and sum rounded to
 *     float64 (no fused multiply-add);
 *   - nearest centre: the smallest distance, ties to the lowest centre index;
 *     a point whose distances are all NaN gets centre 0 and distance +inf;
 *   - centre update: the points are cut into chunks of 4096 consecutive
 *     indices; per chunk the coordinates of a centre's points are summed in
 *     increasing index from 0, the chunk sums (0 for a chunk without its
 *     points) are added in chunk order from 0, then one division by the
 *     count; a centre with no assigned point keeps its coordinates.
 *
 * Conventions as in lma.h: DEVICE pointers unless marked (host), row-major,
 * caller-owned buffers, work ordered on the given stream, status codes with
 * lma_last_error().
 */
#ifndef LMA_PART_H
#define LMA_PART_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "lma.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Nearest centre of each of n points.  P [n][d], C [k][d]; label [n] receives
 * the centre index, dist2 [n] (or NULL) the squared distance to it.
 * 1 <= d <= 64, k >= 1, n >= 0.  Errors: LMA_E_ARG, LMA_E_HIP.
 */
lma_status lma_kmeans_assign(const double *P, int64_t n, int32_t d, const double *C, int32_t k, int32_t *label,
                             double *dist2, hipStream_t stream);

/*
 * Centre update: C [k][d] (in/out) becomes the mean of the points with each
 * label; count [k] (or NULL) receives the number of points per centre.  A
 * point whose label lies outside 0..k-1 counts for no centre.  Uses a
 * transient device block of about 8*k*(d+1) bytes per 4096 points (at most
 * 1 GiB at once) and synchronises the stream before returning it.
 * Errors: LMA_E_ARG, LMA_E_HIP, LMA_E_NOMEM.
 */
lma_status lma_kmeans_update(const double *P, int64_t n, int32_t d, const int32_t *label, int32_t k, double *C,
                             int64_t *count, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the centre
 * update of lma_kmeans_update with the same arguments and the same result bit
 * for bit, but its partial sums live in a fixed 16 MiB scratch array that the
 * library holds on each GPU until the process ends, and it never allocates,
 * frees or synchronises (work is only enqueued on the stream).  Needs
 * 24*k*d + 8*k <= 16 MiB (k*d up to about 690000); larger sizes are rejected
 * with LMA_E_ARG.  Every call on one GPU shares that GPU's scratch: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * ordered by the caller.  Errors: LMA_E_ARG, LMA_E_HIP.
 */
lma_status lma_kmeans_update_noalloc(const double *P, int64_t n, int32_t d, const int32_t *label, int32_t k,
                                     double *C, int64_t *count, hipStream_t stream);

/*
 * Lloyd's iteration: iters rounds of (assign, update) starting from the
 * centres in C (in/out), then a final assignment into label [n] (and dist2
 * [n] or NULL) against the final centres.  iters >= 0.  Synchronises the
 * stream once per round (the centre update).
 * Errors: LMA_E_ARG, LMA_E_HIP, LMA_E_NOMEM.
 */
lma_status lma_kmeans(const double *P, int64_t n, int32_t d, double *C, int32_t k, int32_t iters, int32_t *label,
                      double *dist2, hipStream_t stream);

/*
 * k-means++ seeding (D^2 sampling) of k centres among the n points P [n][d].
 * The first centre is point floor(rand[0] * n / 2^32); centre j >= 1 is drawn
 * with probability proportional to each point's squared distance to its
 * nearest centre so far, using integer weights: with e the binary exponent of
 * the largest such distance (max = f 2^e, 1/2 <= f < 1) and
 * W = 63 - bitlength(n), weight_i = floor(dist_i * 2^(W - e)); with T their sum,
 * the centre is the first point whose running weight sum exceeds
 * floor(rand[j] * T / 2^32) (if T = 0, point floor(rand[j] * n / 2^32)).
 * Integer sums make the draw independent of the summation order.
 * rand (host) [k]: the caller's random 32-bit integers.  C [k][d] receives
 * the centres (copies of the drawn points), index [k] (device, or NULL) their
 * point indices.  Points must be finite.  1 <= k <= 65536, n >= 1.
 * Synchronises the stream.  Errors: LMA_E_ARG, LMA_E_HIP, LMA_E_NOMEM.
 */
lma_status lma_kmeans_seed(const double *P, int64_t n, int32_t d, int32_t k, const uint32_t *rand, double *C,
                           int64_t *index, hipStream_t stream);

/*
 * Capacity-bounded assignment: label [n] receives a centre for every point
 * such that every centre holds between lo and hi points (requires
 * 0 <= lo <= hi, hi >= 1, k*lo <= n <= k*hi).
 *   Upper bound, in rounds: every point without a centre proposes to its
 *   nearest centre among those holding fewer than hi points; a centre with
 *   room for r more points accepts all its proposers if they are at most r,
 *   else its r nearest (smallest squared distance, ties to the lower point
 *   index).  At most k + 1 rounds.
 *   Lower bound, for each centre c holding fewer than lo points, in
 *   increasing c: the point nearest to c (ties to the lower index) among the
 *   points of centres that hold more than lo moves to c, until c holds lo.
 * Distances and nearest centres as in lma_kmeans_assign; every decision is
 * exact, so the labels equal a sequential evaluation of these rules bit for
 * bit.  count [k] (device, or NULL) receives the block sizes, *rounds (host,
 * or NULL) the number of proposal rounds.  Points and centres must be finite.
 * Synchronises the stream once per round.
 * Errors: LMA_E_ARG, LMA_E_HIP, LMA_E_NOMEM.
 */
lma_status lma_bounded_assign(const double *P, int64_t n, int32_t d, const double *C, int32_t k, int64_t lo,
                              int64_t hi, int32_t *label, int64_t *count, int32_t *rounds, hipStream_t stream);

/*
 * The block partition of training inputs X [n][d] and test inputs U [n_u][d]
 * into M blocks (section "Low-Rank-cum-Markov Approximation"):
 *   1. k-means++ seeding of M centres (lma_kmeans_seed with rand (host) [M]);
 *   2. iters rounds of Lloyd's iteration (lma_kmeans);
 *   3. capacity-bounded assignment of X with block sizes in [lo, hi]
 *      (lma_bounded_assign);
 *   4. block centres = the mean of each block's points (lma_kmeans_update);
 *   5. block order = the chain of lma_chain_order through the block centres:
 *      block m is the chain's m-th centre;
 *   6. every test point goes to the block of its nearest block centre;
 *   7. perm [n] (device) lists the training points block by block, the points
 *      of a block in increasing index (X[perm] is block-contiguous);
 *      block_ptr (host) [M+1] the block boundaries; u_perm [n_u] (device) and
 *      u_block_ptr (host) [M+1] the same for the test points (NULL when
 *      n_u = 0; empty test blocks are possible).
 * centres [M][d] (device, or NULL) receives the block centres in block order.
 * lma_fit needs every block non-empty: take lo >= 1.  Points must be finite.
 * Synchronises the stream.
 * Errors: LMA_E_ARG, LMA_E_HIP, LMA_E_NOMEM.
 */
lma_status lma_partition(const double *X, int64_t n, const double *U, int64_t n_u, int32_t d, int32_t M, int64_t lo,
                         int64_t hi, int32_t iters, const uint32_t *rand, int64_t *perm, int64_t *block_ptr,
                         int64_t *u_perm, int64_t *u_block_ptr, double *centres, hipStream_t stream);

/*
 * Order of the blocks along the Markov chain (host function, no device work):
 * LMA couples each block with the next B blocks in the given order, so
 * neighbouring blocks should be close.  C [k][d] (host) are the block centres;
 * order [k] (host) receives a permutation of 0..k-1: it starts at the centre
 * farthest from the mean of the centres (the mean summed over the centres in
 * index order, then divided by k) and moves each time to the nearest centre
 * not yet visited.  Distances are evaluated as in the assignment above
 * (coordinates in order, no fused multiply-add; ties to the lowest index).
 * 1 <= d <= 64, k >= 1.  Errors: LMA_E_ARG.
 */
lma_status lma_chain_order(const double *C, int32_t k, int32_t d, int32_t *order);

#ifdef __cplusplus
}
#endif

#endif /* LMA_PART_H */
