// Small kernels around the engine: input scaling, the global summary
// finalisation, the |S|x|S| global solve, and the per-test-point prediction
// combine.
#include "misc.h"

namespace lma {

__global__ void k_scale(const double* __restrict__ X, int64_t n, int d, InvEll ie, double* __restrict__ o64,
                        float* __restrict__ o32) {
  const int64_t tot = n * d;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(i % d);
    const double v = X[i] * ie.v[t];
    if (o64) o64[i] = v;
    if (o32) o32[i] = (float)v;
  }
}

__global__ void k_center(const double* __restrict__ y, int64_t n, double mu, double* __restrict__ c64,
                         float* __restrict__ c32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = y[i] - mu;
    if (c64) c64[i] = v;
    if (c32) c32[i] = (float)v;
  }
}

__global__ void k_cast(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

__global__ void k_zero(double* __restrict__ a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0.0;
}

__device__ inline double se_kernel(const double* a, const double* b, int d, double sf2) {
  double s = 0.0;
  for (int t = 0; t < d; ++t) {
    const double df = a[t] - b[t];
    s += df * df;
  }
  return sf2 * exp(-0.5 * s);
}

// Sum the per-group partial tiles in group order and assemble
//   Sigma_ddot_SS = Sigma_SS + sum_m Z_m^T Z_m   (full symmetric, identity on padding)
//   y_ddot_S      = sum_m Z_m^T z_m
//   q             = sum_m z_m^T z_m
// Tile t = a(a+1)/2 + b of the (Ts+1) x (Ts+1) lower tile grid; tile row/col Ts
// is the centred-output row.
__global__ __launch_bounds__(256) void k_finalize_summary(SummaryArgs a) {
  const int t = blockIdx.x;
  int ta = 0;
  while ((ta + 1) * (ta + 2) / 2 <= t) ++ta;
  const int tb = t - ta * (ta + 1) / 2;
  for (int idx = threadIdx.x; idx < 128 * 128; idx += blockDim.x) {
    const int r = idx >> 7, c = idx & 127;
    double v = 0.0;
    for (int g = 0; g < a.groups; ++g) v += a.partial[((int64_t)g * a.ntile + t) * 16384 + idx];
    if (ta < a.Ts) {
      if (ta == tb && c > r) continue;
      const int R = ta * 128 + r, C = tb * 128 + c;
      double k;
      if (R < a.s && C < a.s)
        k = se_kernel(a.Ss + (int64_t)R * a.d, a.Ss + (int64_t)C * a.d, a.d, a.sf2) + (R == C ? a.sn2 : 0.0);
      else
        k = (R == C) ? 1.0 : 0.0;
      a.Sdd[(int64_t)R * a.sp + C] = k + v;
      a.Sdd[(int64_t)C * a.sp + R] = k + v;
    } else if (r == 0) {
      if (tb < a.Ts)
        a.ydd[tb * 128 + c] = (tb * 128 + c < a.s) ? v : 0.0;
      else if (c == 0)
        a.qsum[0] = v;
    }
  }
}

// Solve Sigma_ddot_SS g = y_ddot_S with its tiled Cholesky factor (inverted
// diagonal tiles), followed by `iters` steps of iterative refinement with the
// float64 matrix.  One workgroup.
__global__ __launch_bounds__(256) void k_global_solve(SolveArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* x = reinterpret_cast<double*>(smem_raw);  // [sp] solution
  double* r = x + a.sp;                             // [sp] residual / work vector
  double* tmp = r + a.sp;                           // [128]
  const int tid = threadIdx.x;
  const int Ts = a.sp / 128;
  for (int i = tid; i < a.sp; i += blockDim.x) x[i] = 0.0;
  __syncthreads();
  for (int it = 0; it <= a.iters; ++it) {
    // residual r = b - A x
    for (int i = tid; i < a.sp; i += blockDim.x) {
      double acc = a.b[i];
      if (it > 0) {
        const double* row = a.A + (int64_t)i * a.sp;
        for (int k = 0; k < a.sp; ++k) acc -= row[k] * x[k];
      }
      r[i] = acc;
    }
    __syncthreads();
    // forward: L z = r (z overwrites r tile by tile)
    for (int ti = 0; ti < Ts; ++ti) {
      const double* Lrow = a.L + (int64_t)64 * 128 * ti * (ti + 1);  // 128*128*ti(ti+1)/2
      const int64_t ld = (int64_t)(ti + 1) * 128;
      if (tid < 128) {
        double acc = r[ti * 128 + tid];
        for (int k = 0; k < ti * 128; ++k) acc -= Lrow[(int64_t)tid * ld + k] * r[k];
        tmp[tid] = acc;
      }
      __syncthreads();
      if (tid < 128) {
        const double* inv = a.inv + (int64_t)ti * 16384;
        double acc = 0.0;
        for (int c = 0; c <= tid; ++c) acc += inv[tid * 128 + c] * tmp[c];
        r[ti * 128 + tid] = acc;
      }
      __syncthreads();
    }
    // backward: L^T w = z (w overwrites r, last tile first)
    for (int ti = Ts - 1; ti >= 0; --ti) {
      if (tid < 128) {
        double acc = r[ti * 128 + tid];
        for (int tk = ti + 1; tk < Ts; ++tk) {
          const double* Lk = a.L + (int64_t)64 * 128 * tk * (tk + 1) + ti * 128;
          const int64_t ld = (int64_t)(tk + 1) * 128;
          for (int c = 0; c < 128; ++c) acc -= Lk[(int64_t)c * ld + tid] * r[tk * 128 + c];
        }
        tmp[tid] = acc;
      }
      __syncthreads();
      if (tid < 128) {
        const double* inv = a.inv + (int64_t)ti * 16384;
        double acc = 0.0;
        for (int c = tid; c < 128; ++c) acc += inv[c * 128 + tid] * tmp[c];
        r[ti * 128 + tid] = acc;
      }
      __syncthreads();
    }
    for (int i = tid; i < a.sp; i += blockDim.x) x[i] += r[i];
    __syncthreads();
  }
  for (int i = tid; i < a.sp; i += blockDim.x) a.g[i] = x[i];
}

// E_u = k_u - G_u (in place in G), mean_u = mu + E_u . g + l_u, |V_u|^2.
// One wave per test point.
__global__ __launch_bounds__(256) void k_pred_E(PredArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (u >= a.n_u) return;
  double* Gu = a.G + u * a.ldG;
  const double* xu = a.Us + u * a.d;
  double am = 0.0, av = 0.0;
  for (int k = lane; k < a.sp; k += 64) {
    const double kv = k < a.s ? se_kernel(xu, a.Ss + (int64_t)k * a.d, a.d, a.sf2) : 0.0;
    const double e = kv - Gu[k];
    Gu[k] = e;
    am += e * a.g[k];
    const double vv = a.VtU[u * a.sp + k];
    av += vv * vv;
  }
  for (int o = 32; o > 0; o >>= 1) {
    am += __shfl_xor(am, o);
    av += __shfl_xor(av, o);
  }
  if (lane == 0) {
    if (a.mean) a.mean[u] = a.mu + am + Gu[a.sp];
    a.vn[u] = av;
  }
}

// xi_u = sum over the windows of u's test block q (m = q-B .. q) of the squared
// whitened residual cross-covariances: all columns of window q, the D_m
// columns of the others.  One wave per test point.
template <typename T>
__global__ __launch_bounds__(256) void k_pred_xi(XiArgs<T> a) {
  const int lane = threadIdx.x & 63;
  const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (u >= a.n_u) return;
  const int q = a.ublk[u];
  double acc = 0.0;
  for (int dl = 0; dl <= a.B && dl <= q; ++dl) {
    const int m = q - dl;
    if (m < a.m0 || m >= a.m1) continue;
    const int64_t ldx = (int64_t)a.Tm[m] * 128;
    const T* row = a.Xbuf + a.Xoff[m] + (u - a.uptr[m]) * ldx;
    const int k0 = dl == 0 ? 0 : a.twm[m] * 128;
    for (int k = k0 + lane; k < ldx; k += 64) {
      const double v = (double)row[k];
      acc += v * v;
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) a.xi[u] = a.accumulate ? a.xi[u] + acc : acc;
}

// var_u = sigma_s^2 + sigma_n^2 - |V_u|^2 - xi_u + |L_ddot^-1 E_u|^2.
__global__ __launch_bounds__(256) void k_pred_var(PredArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (u >= a.n_u) return;
  const double* Tu = a.G + u * a.ldG;
  double acc = 0.0;
  for (int k = lane; k < a.sp; k += 64) acc += Tu[k] * Tu[k];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0 && a.var) a.var[u] = a.sf2 + a.sn2 - a.vn[u] - a.xi[u] + acc;
}

// ---------------------------------------------------------------------------
static inline int nblk(int64_t n, int per) { return (int)std::min<int64_t>((n + per - 1) / per, 65535 * 8); }

void launch_scale(const double* X, int64_t n, int d, const InvEll& ie, double* o64, float* o32, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale, dim3(nblk(n * d, 256)), dim3(256), 0, st, X, n, d, ie, o64, o32);
}
void launch_center(const double* y, int64_t n, double mu, double* c64, float* c32, hipStream_t st) {
  hipLaunchKernelGGL(k_center, dim3(nblk(n, 256)), dim3(256), 0, st, y, n, mu, c64, c32);
}
void launch_cast(const double* a, float* b, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_cast, dim3(nblk(n, 256)), dim3(256), 0, st, a, b, n);
}
void launch_zero(double* a, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero, dim3(nblk(n, 256)), dim3(256), 0, st, a, n);
}
void launch_finalize_summary(const SummaryArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_summary, dim3(a.ntile), dim3(256), 0, st, a);
}
size_t global_solve_lds(int sp) { return sizeof(double) * (size_t)(2 * sp + 128); }
void launch_global_solve(const SolveArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_global_solve, dim3(1), dim3(256), global_solve_lds(a.sp), st, a);
}
void launch_pred_E(const PredArgs& a, hipStream_t st) {
  if (a.n_u <= 0) return;
  hipLaunchKernelGGL(k_pred_E, dim3((unsigned)((a.n_u + 3) / 4)), dim3(256), 0, st, a);
}
void launch_pred_var(const PredArgs& a, hipStream_t st) {
  if (a.n_u <= 0) return;
  hipLaunchKernelGGL(k_pred_var, dim3((unsigned)((a.n_u + 3) / 4)), dim3(256), 0, st, a);
}
template <typename T>
void launch_pred_xi(const XiArgs<T>& a, hipStream_t st) {
  if (a.n_u <= 0) return;
  hipLaunchKernelGGL(k_pred_xi<T>, dim3((unsigned)((a.n_u + 3) / 4)), dim3(256), 0, st, a);
}
template void launch_pred_xi<double>(const XiArgs<double>&, hipStream_t);
template void launch_pred_xi<float>(const XiArgs<float>&, hipStream_t);

hipError_t misc_init() {
  return hipFuncSetAttribute((const void*)k_global_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)global_solve_lds(8192));
}

}  // namespace lma
