/*
 * lma_part.h -- C ABI of the clustering steps that partition the data into
 * blocks (gfx950).
 *
 * LMA needs the training and test inputs partitioned into M blocks (section
 * "Low-Rank-cum-Markov Approximation"; the paper leaves the scheme to a
 * clustering method of earlier work).  The library takes the partition as an
 * input (block_ptr in lma.h); these entry points run the data-parallel part
 * of a k-means partitioner on the GPU: the nearest-centre assignment of every
 * point and the centre update of Lloyd's iteration.  Seeding, a bound on the
 * block sizes and the order of the blocks along the Markov chain are left to
 * the caller.
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
