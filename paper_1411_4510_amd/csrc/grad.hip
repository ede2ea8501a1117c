// Device kernels of the log-marginal-likelihood adjoint (gfx950).
#include "grad.h"
#include "mfma_core.h"
#include "misc.h"

#include <type_traits>

namespace lma {

// One 128 x 128 adjoint tile: signed tile GEMMs on the matrix cores, then the
// epilogue adds the rank-one / explicit terms, regenerates the covariance tile
// from LDS-staged coordinates and contracts it with its d+2 derivatives.
template <typename TX>
__global__ __launch_bounds__(NT) void k_dcontract(DcArgs<TX> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[NT / 64][MAX_D + 2];
  const int logical = xcd_logical(blockIdx.x, gridDim.x);
  if (logical >= a.nitems) return;
  const DcItem it = a.items[logical];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const int d = a.d;

  typename Mfma<double>::acc acc[4][4];
  zero_acc<double>(acc);
  for (int t = it.x0; t < it.x1; ++t) {
    const GemmTerm<TX> tm = a.xterms[t];
    wave_gemm<TX, double>(acc, tm.a, tm.lda, tm.anr, tm.b, tm.ldb, tm.bnr, tm.k0, tm.k1, wr * 64, wc * 64, lane);
  }
  for (int t = it.t0; t < it.tneg; ++t) {
    const GemmTerm<double> tm = a.terms[t];
    wave_gemm<double, double>(acc, tm.a, tm.lda, tm.anr, tm.b, tm.ldb, tm.bnr, tm.k0, tm.k1, wr * 64, wc * 64,
                              lane);
  }
  if (it.x1 > it.x0 || it.tneg > it.t0) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] = -acc[p][q];
  }
  for (int t = it.tneg; t < it.t1; ++t) {
    const GemmTerm<double> tm = a.terms[t];
    wave_gemm<double, double>(acc, tm.a, tm.lda, tm.anr, tm.b, tm.ldb, tm.bnr, tm.k0, tm.k1, wr * 64, wc * 64,
                              lane);
  }

  double* xr = reinterpret_cast<double*>(smem_raw);  // [d][TB]
  double* xc = xr + d * TB;                          // [d][TB]
  for (int idx = tid; idx < TB * d; idx += NT) {
    const int r = idx / d, q = idx - r * d;
    xr[q * TB + r] = r < it.nr ? it.xr[(int64_t)r * d + q] : 0.0;
    xc[q * TB + r] = r < it.nc ? it.xc[(int64_t)r * d + q] : 0.0;
  }
  __syncthreads();

  // squared distances of the lane's 64 entries, one length-scale at a time
  double dist[4][4][4];
#pragma unroll
  for (int rs = 0; rs < 4; ++rs)
#pragma unroll
    for (int cs = 0; cs < 4; ++cs)
#pragma unroll
      for (int v = 0; v < 4; ++v) dist[rs][cs][v] = 0.0;
  for (int q = 0; q < d; ++q) {
    double cv[4];
#pragma unroll
    for (int cs = 0; cs < 4; ++cs) cv[cs] = xc[q * TB + wc * 64 + cs * 16 + (lane & 15)];
#pragma unroll
    for (int rs = 0; rs < 4; ++rs)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double rv = xr[q * TB + wr * 64 + rs * 16 + Mfma<double>::row(lane, v)];
#pragma unroll
        for (int cs = 0; cs < 4; ++cs) {
          const double df = rv - cv[cs];
          dist[rs][cs][v] += df * df;
        }
      }
  }
  // pass 1: e_ij = wt * A_ij * k_ij (kept in acc), signal and noise sums
  const bool same_diag = it.kind == DC_SAME && it.diag;
  const double sf2 = a.sf2, sn2 = a.sn2;
  double gs = 0.0, gn = 0.0;
#pragma unroll
  for (int rs = 0; rs < 4; ++rs)
#pragma unroll
    for (int cs = 0; cs < 4; ++cs)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 64 + rs * 16 + Mfma<double>::row(lane, v);
        const int col = wc * 64 + cs * 16 + (lane & 15);
        double e = 0.0;
        if (row < it.nr && col < it.nc) {
          double val = acc[rs][cs][v];
#pragma unroll
          for (int r = 0; r < 2; ++r)
            if (r < it.nr1) val += it.r1s[r] * it.r1a[r][row] * it.r1b[r][col];
#pragma unroll
          for (int x = 0; x < 2; ++x)
            if (x < it.nex) val += it.exs[x] * it.ex[x][(int64_t)row * it.exld[x] + col];
          e = it.wt * val * (sf2 * exp(-0.5 * dist[rs][cs][v]));
          gs += e;
          if (same_diag && row == col) gn += it.wt * val * sn2;
        }
        acc[rs][cs][v] = e;
      }

  // pass 2: one length-scale at a time
  for (int q = 0; q < d; ++q) {
    double cv[4];
#pragma unroll
    for (int cs = 0; cs < 4; ++cs) cv[cs] = xc[q * TB + wc * 64 + cs * 16 + (lane & 15)];
    double s = 0.0;
#pragma unroll
    for (int rs = 0; rs < 4; ++rs)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double rv = xr[q * TB + wr * 64 + rs * 16 + Mfma<double>::row(lane, v)];
#pragma unroll
        for (int cs = 0; cs < 4; ++cs) {
          const double df = rv - cv[cs];
          s += acc[rs][cs][v] * df * df;
        }
      }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[w][q] = s;
  }
  for (int o = 32; o > 0; o >>= 1) {
    gs += __shfl_xor(gs, o);
    gn += __shfl_xor(gn, o);
  }
  if (lane == 0) {
    red[w][d] = gs;
    red[w][d + 1] = gn;
  }
  __syncthreads();
  if (tid < d + 2)
    a.partial[(int64_t)logical * (d + 2) + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

__global__ __launch_bounds__(NT) void k_reduce_partials(const double* __restrict__ partial, int64_t nitems,
                                                        int ncomp, double* __restrict__ out) {
  __shared__ double red[NT];
  const int q = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int64_t i = tid; i < nitems; i += NT) s += partial[i * ncomp + q];
  red[tid] = s;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) out[q] = red[0];
}

__global__ void k_sig_ss(const double* __restrict__ Ss, int s, int sp, int d, double sf2, double sn2,
                         double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)sp * sp) return;
  const int a = (int)(idx / sp), b = (int)(idx - (int64_t)a * sp);
  double v;
  if (a < s && b < s) {
    double dist = 0.0;
    for (int q = 0; q < d; ++q) {
      const double df = Ss[(int64_t)a * d + q] - Ss[(int64_t)b * d + q];
      dist += df * df;
    }
    v = sf2 * exp(-0.5 * dist) + (a == b ? sn2 : 0.0);
  } else {
    v = a == b ? 1.0 : 0.0;
  }
  out[idx] = v;
}

__global__ void k_lincomb(double* __restrict__ out, const double* __restrict__ x, double alpha,
                          const double* __restrict__ y, double beta, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = alpha * x[i] + beta * y[i];
}

__global__ void k_uvec(double* __restrict__ u, const double* __restrict__ g, const double* __restrict__ hT,
                       int64_t ldh, int nx, int sp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nx * sp) return;
  const int x = (int)(i / sp), t = (int)(i - (int64_t)x * sp);
  u[i] = g[t] - hT[(int64_t)t * ldh + x];
}

__global__ void k_sum_groups(double* __restrict__ out, const double* __restrict__ a, const double* __restrict__ b,
                             const double* __restrict__ parts, int ng, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = a[i] - b[i];
  for (int k = 0; k < ng; ++k) s += parts[(int64_t)k * n + i];
  out[i] = s;
}

static inline int pad8(int n) { return ((n + 7) / 8) * 8; }
static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename TX>
void launch_dcontract(const DcArgs<TX>& a, hipStream_t st) {
  if (a.nitems <= 0) return;
  const size_t lds = 2 * (size_t)a.d * TB * sizeof(double);
  hipLaunchKernelGGL(k_dcontract<TX>, dim3(pad8(a.nitems)), dim3(NT), lds, st, a);
}

void launch_reduce_partials(const double* partial, int64_t nitems, int ncomp, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(ncomp), dim3(NT), 0, st, partial, nitems, ncomp, out);
}

void launch_sig_ss(const double* Ss, int s, int sp, int d, double sf2, double sn2, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sig_ss, dim3(nblk((int64_t)sp * sp)), dim3(256), 0, st, Ss, s, sp, d, sf2, sn2, out);
}

void launch_lincomb(double* out, const double* x, double alpha, const double* y, double beta, int64_t n,
                    hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_lincomb, dim3(nblk(n)), dim3(256), 0, st, out, x, alpha, y, beta, n);
}

void launch_uvec(double* u, const double* g, const double* hT, int64_t ldh, int nx, int sp, hipStream_t st) {
  if (nx <= 0) return;
  hipLaunchKernelGGL(k_uvec, dim3(nblk((int64_t)nx * sp)), dim3(256), 0, st, u, g, hT, ldh, nx, sp);
}

void launch_sum_groups(double* out, const double* a, const double* b, const double* parts, int ng, int64_t n,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_sum_groups, dim3(nblk(n)), dim3(256), 0, st, out, a, b, parts, ng, n);
}

hipError_t grad_init() {
  const int lds = (int)(2 * MAX_D * TB * sizeof(double));
  hipError_t e = hipFuncSetAttribute((const void*)k_dcontract<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_dcontract<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

template void launch_dcontract<double>(const DcArgs<double>&, hipStream_t);
template void launch_dcontract<float>(const DcArgs<float>&, hipStream_t);

}  // namespace lma
