// SE-ARD kernel-matrix times vector on tiles (kvec.hip).
//
// An item is a tile of up to 128 row points; it runs over a list of column
// tiles (up to 128 column points each, with one or two vectors) and forms
//   acc0[r] = sum_c k(x_r, x_c) v0[c],   acc1[r] = sum_c k(x_r, x_c) v1[c]
// with k the SE-ARD covariance (no noise) of length-scaled coordinates.  The
// squared distances come from |x|^2 + |y|^2 - 2 x.y with the cross term on the
// float64 matrix cores; exp and the vector products run on the vector units.
// A per-use epilogue turns the two sums into the output rows.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lma {

enum KvMode : int32_t {
  KV_CG = 0,    // out0[r] = base0[r] - acc0                    (c' = c - K_XS g)
  KV_MEAN = 1,  // out0[r] = mu + acc0 - acc1 - vt_r . h0        (predictive mean)
  KV_KMV = 2,   // out0[r] = base0[r] - (acc0 + sn2 self0[r] - vt_r . h0), and with flag
                // out1[r] = base0[r] - (acc1 + sn2 self1[r] - vt_r . h1); padding rows get 0
};

struct KvCol {
  const double* x;   // coordinates of the column points [nc][d]
  const double* v0;  // first vector over the columns (null: zero)
  const double* v1;  // second vector (null: zero)
  int32_t nc;
  int32_t pad_;
};

struct KvItem {
  const double* x;      // coordinates of the row points [nr][d]
  const double* base0;  // KV_CG: c of the rows; KV_KMV: right-hand side c' of the rows
  const double* vt;     // whitened support rows of the row points (row r at vt + r*sp) or null
  const double* h0;
  const double* h1;
  const double* self0;
  const double* self1;
  double* out0;
  double* out1;
  int32_t nr;
  int32_t c0, c1;       // column tiles [c0, c1) of the column list
  int32_t flag;         // KV_KMV: 1 when out1 is wanted (rows in W_m)
};

struct KvArgs {
  const KvItem* items;
  const KvCol* cols;
  int32_t nitems;
  int32_t mode;
  int32_t d, sp;
  double sf2, sn2, mu;
};

void launch_kvec(const KvArgs& a, hipStream_t st);
// hq[q] = sum_{dl=0..min(B,q)} hJ[q-dl] - sum_{dl=1..min(B,q)} hW[q-dl]   ([M][sp])
void launch_hq(const double* hJ, const double* hW, double* hq, int M, int B, int sp, hipStream_t st);
hipError_t kvec_init();

}  // namespace lma
