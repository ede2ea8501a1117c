/*
 * lma_ds.h -- C ABI of the warm-start network (gfx950) that predicts starting
 * log-hyperparameters for the LMA likelihood from a dataset.
 *
 * The network is a deep-sets regressor: a per-point encoder of two ReLU
 * layers of width 256 on 17 per-point features, the mean over the points of a
 * dataset, and a head of one ReLU layer of width 256 and a linear layer to 10
 * outputs (log l_1..log l_8, log sigma_s^2, log sigma_n^2, for inputs in the
 * unit cube and standardised outputs).  Per-point features (float32, row-major
 * [n][17]): x_1..x_8 (zero beyond the input dimension d), (y - mean(y)) /
 * std(y), and eight dimension-mask entries (1 for k < d, else 0).
 *
 * Arithmetic: float32 master weights; products use their bfloat16 roundings
 * on the matrix cores with float32 accumulation; the per-point inputs of the
 * two encoder layers and the per-point gradients of the backward pass are
 * rounded to bfloat16 where they enter a product; bias, ReLU, mean and the
 * head are float32.  Training loss: per dataset the mean squared error over
 * its valid outputs (given by a 0/1 mask), averaged over the datasets of the
 * batch; Adam on the master weights.
 *
 * Parameter vector (float32, host or device as stated): W1 [256][17], b1
 * [256], W2 [256][256], b2 [256], W3 [256][256], b3 [256], W4 [10][256],
 * b4 [10], concatenated in that order (LMA_DS_NPARAM entries).
 *
 * Batches: nsets datasets whose points occupy rows set_ptr[b] ..
 * set_ptr[b] + set_n[b] - 1 of the feature array, with set_ptr[b] a multiple
 * of 128 (rows between sets are padding and are never read); set_ptr[nsets]
 * rows in total.  Conventions as in lma.h: device pointers unless marked
 * (host), work ordered on the given stream, status codes, lma_last_error().
 */
#ifndef LMA_DS_H
#define LMA_DS_H
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lma.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LMA_DS_NPARAM 138762
#define LMA_DS_NFEAT 17
#define LMA_DS_NOUT 10

typedef struct lma_ds lma_ds;

/* Network state with workspace for up to max_rows feature rows (set_ptr[nsets])
 * and max_sets datasets per call; parameters are zero until set. */
lma_status lma_ds_create(int64_t max_rows, int64_t max_sets, lma_ds **out);
void lma_ds_free(lma_ds *ds);

/* Copy the master parameters in / out (host [LMA_DS_NPARAM]); setting them
 * also resets the Adam moments and step count.  Synchronous. */
lma_status lma_ds_set_params(lma_ds *ds, const float *params);
lma_status lma_ds_get_params(lma_ds *ds, float *params);

/* Per-point features of one dataset from its inputs X [n][d] (float64, d <= 8)
 * and outputs y [n] (float64), written to feats [n][17] (float32); the mean
 * and standard deviation of y use a small scratch area of the state. */
lma_status lma_ds_features(lma_ds *ds, const double *X, const double *y, int64_t n, int32_t d, float *feats,
                           hipStream_t stream);

/* Forward pass: out [nsets][10] (float32).  set_ptr (host [nsets+1]) and set_n
 * (host [nsets]) as described above.  Keeps the activations for a following
 * lma_ds_backward on the same state. */
lma_status lma_ds_forward(lma_ds *ds, int64_t nsets, const int64_t *set_ptr, const int64_t *set_n,
                          const float *feats, float *out, hipStream_t stream);

/* Backward pass of the last forward: gradient of the batch loss against
 * labels [nsets][10] with masks [nsets][10] (float32, device).  The gradient
 * is kept in the state (for lma_ds_adam) and copied to grad (device
 * [LMA_DS_NPARAM]) if not NULL; the loss is written to *loss (host) if not
 * NULL (synchronises the stream). */
lma_status lma_ds_backward(lma_ds *ds, const float *labels, const float *masks, float *grad, double *loss,
                           hipStream_t stream);

/* One Adam step on the master weights with the kept gradient (step counter
 * advanced by the library; bias corrections use it). */
lma_status lma_ds_adam(lma_ds *ds, float lr, float beta1, float beta2, float eps, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* LMA_DS_H */
