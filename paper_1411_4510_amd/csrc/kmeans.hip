// k-means steps of the block partitioner on gfx950 (include/lma_part.h).
//
// Nearest-centre assignment: one thread per point.  The centres are read with
// wave-uniform loads (every lane of a wave reads the same centre entry), eight
// centres per pass, so a lane keeps eight running sums in registers and reads
// each of its point's coordinates once per pass.  Each distance is summed over
// the coordinates in increasing order with separately rounded products and
// sums (contraction into fused multiply-adds is switched off), so the result
// is the same bit for bit as any plain evaluation in that order.
//
// Centre update: one thread per (centre, coordinate) walks all points in
// increasing index and adds the coordinate of those with its label (the label
// read is wave-uniform), then divides once by the count.  Every sum has a
// fixed order, so the update does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lma_part.h"
#include "misc.h"
#include "runtime.h"

namespace lma {
namespace part {

constexpr int NTA = 256;   // threads per workgroup, assignment
constexpr int CG = 8;      // centres per pass
constexpr int NTU = 64;    // threads per workgroup, update
constexpr int MAX_K = 65536;

__global__ __launch_bounds__(NTA) void k_km_assign(const double* __restrict__ P, int64_t n, int d,
                                                   const double* __restrict__ C, int k, int32_t* __restrict__ label,
                                                   double* __restrict__ dist2) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * NTA + threadIdx.x;
  if (i >= n) return;
  const double* p = P + i * d;
  double best = INFINITY;
  int arg = 0;
  for (int c0 = 0; c0 < k; c0 += CG) {
    const int nc = k - c0 < CG ? k - c0 : CG;
    double acc[CG];
#pragma unroll
    for (int j = 0; j < CG; ++j) acc[j] = 0.0;
    const double* cb = C + (int64_t)c0 * d;
    for (int t = 0; t < d; ++t) {
      const double x = p[t];
#pragma unroll
      for (int j = 0; j < CG; ++j) {
        if (j < nc) {
          const double df = x - cb[j * d + t];
          const double sq = df * df;
          acc[j] = acc[j] + sq;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < CG; ++j)
      if (j < nc && acc[j] < best) {
        best = acc[j];
        arg = c0 + j;
      }
  }
  label[i] = arg;
  if (dist2) dist2[i] = best;
}

__global__ __launch_bounds__(NTU) void k_km_update(const double* __restrict__ P, int64_t n, int d,
                                                   const int32_t* __restrict__ label, int k, double* __restrict__ C,
                                                   int64_t* __restrict__ count) {
  const int64_t e = (int64_t)blockIdx.x * NTU + threadIdx.x;
  if (e >= (int64_t)k * d) return;
  const int c = (int)(e / d), t = (int)(e - (int64_t)c * d);
  double s = 0.0;
  int64_t cnt = 0;
  int64_t i = 0;
  for (; i + 8 <= n; i += 8) {
    int32_t lb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) lb[j] = label[i + j];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (lb[j] == c) {
        s = s + P[(i + j) * d + t];
        ++cnt;
      }
  }
  for (; i < n; ++i)
    if (label[i] == c) {
      s = s + P[i * d + t];
      ++cnt;
    }
  if (cnt > 0) C[e] = s / (double)cnt;
  if (count && t == 0) count[c] = cnt;
}

}  // namespace part
}  // namespace lma

namespace {

using lmart::Err;

void check_shape(const double* P, int64_t n, int32_t d, int32_t k) {
  if (n < 0) throw Err{LMA_E_ARG, "n < 0"};
  if (d < 1 || d > lma::MAX_D) throw Err{LMA_E_ARG, "need 1 <= d <= 64"};
  if (k < 1 || k > lma::part::MAX_K) throw Err{LMA_E_ARG, "need 1 <= k <= 65536"};
  if (n > 0 && !P) throw Err{LMA_E_ARG, "P is NULL"};
}

void assign(const double* P, int64_t n, int32_t d, const double* C, int32_t k, int32_t* label, double* dist2,
            hipStream_t st) {
  if (n == 0) return;
  const int64_t nb = (n + lma::part::NTA - 1) / lma::part::NTA;
  if (nb > 0x7fffffff) throw Err{LMA_E_ARG, "too many points"};
  hipLaunchKernelGGL(lma::part::k_km_assign, dim3((unsigned)nb), dim3(lma::part::NTA), 0, st, P, n, (int)d, C, (int)k,
                     label, dist2);
  HIPCHK(hipGetLastError());
}

void update(const double* P, int64_t n, int32_t d, const int32_t* label, int32_t k, double* C, int64_t* count,
            hipStream_t st) {
  const int64_t nt = (int64_t)k * d;
  const int64_t nb = (nt + lma::part::NTU - 1) / lma::part::NTU;
  hipLaunchKernelGGL(lma::part::k_km_update, dim3((unsigned)nb), dim3(lma::part::NTU), 0, st, P, n, (int)d, label,
                     (int)k, C, count);
  HIPCHK(hipGetLastError());
}

template <class F>
lma_status guard(F&& f) {
  lmart::set_last_error("");
  try {
    f();
    return LMA_OK;
  } catch (const Err& e) {
    lmart::set_last_error(e.msg);
    return e.st;
  } catch (const std::bad_alloc&) {
    lmart::set_last_error("host allocation failed");
    return LMA_E_NOMEM;
  } catch (const std::exception& e) {
    lmart::set_last_error(std::string("internal error: ") + e.what());
    return LMA_E_INTERNAL;
  }
}

}  // namespace

extern "C" {

lma_status lma_kmeans_assign(const double* P, int64_t n, int32_t d, const double* C, int32_t k, int32_t* label,
                             double* dist2, hipStream_t stream) {
  return guard([&] {
    check_shape(P, n, d, k);
    if (n > 0 && (!C || !label)) throw Err{LMA_E_ARG, "NULL array"};
    assign(P, n, d, C, k, label, dist2, stream);
  });
}

lma_status lma_kmeans_update(const double* P, int64_t n, int32_t d, const int32_t* label, int32_t k, double* C,
                             int64_t* count, hipStream_t stream) {
  return guard([&] {
    check_shape(P, n, d, k);
    if (!C || (n > 0 && !label)) throw Err{LMA_E_ARG, "NULL array"};
    update(P, n, d, label, k, C, count, stream);
  });
}

lma_status lma_kmeans(const double* P, int64_t n, int32_t d, double* C, int32_t k, int32_t iters, int32_t* label,
                      double* dist2, hipStream_t stream) {
  return guard([&] {
    check_shape(P, n, d, k);
    if (iters < 0) throw Err{LMA_E_ARG, "iters < 0"};
    if (!C || (n > 0 && !label)) throw Err{LMA_E_ARG, "NULL array"};
    for (int32_t it = 0; it < iters; ++it) {
      assign(P, n, d, C, k, label, nullptr, stream);
      if (n > 0) update(P, n, d, label, k, C, nullptr, stream);
    }
    assign(P, n, d, C, k, label, dist2, stream);
  });
}

}  // extern "C"
