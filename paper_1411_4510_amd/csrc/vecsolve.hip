// Vector solves with the stored window factors and the predictive mean.
//
// With g = Sigma_ddot_SS^-1 y_ddot_S and beta_X = R_X^-1 (c_X - K_XS g) for the
// windows X = J_m and the separators X = W_m, the predictive mean of Eq. (3)
// for u in test block q is
//   mu + k_u^T g + sum_{m=q-B..q} R_{u,J_m} beta_{J_m} - sum_{m=q-B..q-1} R_{u,W_m} beta_{W_m}.
// (Woodbury on Sigma_bar_DD = Q + R_bar and the signed window sum of
// R_bar_DD^-1 that the banded factor of Lemma 1 gives; the separator term of
// window q cancels against its own leading block.)  Only vector solves are
// needed, so they run in float64 arithmetic even on float32 factors.  The
// forward half is read off the whitened right-hand sides the factorisation
// already produced.  In mixed precision one refinement of beta against the
// float64 residual covariance and one global correction of g (whose residual
// is L_SS (sum_m V_{J_m} beta_{J_m} - V_{W_m} beta_{W_m}) - Sigma_SS g)
// restore float64-level accuracy of the mean.
#include "engine.h"
#include "misc.h"

namespace lma {

__device__ inline int64_t win_point(const WinTab& w, int m, int r, bool& valid) {
  const int tw = w.tw[m];
  if (r < tw * TB) {
    valid = r < w.wlen[m];
    return w.wstart[m] + r;
  }
  const int rr = r - tw * TB;
  valid = rr < w.dlen[m];
  return w.dstart[m] + rr;
}

__device__ inline int64_t jp_off(int i) { return (int64_t)TB * TB * i * (i + 1) / 2; }

__device__ inline double sqd(const double* a, const double* b, int d) {
  double s = 0.0;
  for (int t = 0; t < d; ++t) {
    const double df = a[t] - b[t];
    s += df * df;
  }
  return s;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ---------------------------------------------------------------------------
// triangular solves of one vector per window (one workgroup of 8 waves per
// window; the panels are streamed once per solve with 16-byte loads)
// ---------------------------------------------------------------------------
constexpr int SOLVE_NT = 512;
constexpr size_t FWD_LDS_MAX = 150 * 1024;  // solved prefix of windows up to 19200 rows in LDS

template <typename TW>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};

// forward, left-looking: t_i = v_i - L_{i,<i} x_{<i}, x_i = L_ii^-1 t_i, x in v.
// xs holds the solved prefix (LDS when it fits, else v itself).
template <typename TW>
__device__ void fwd_solve(const TW* base, const TW* inv, double* v, int nt, double* xs, double* t) {
  typedef typename Vec16<TW>::type VT;
  constexpr int NV = Vec16<TW>::n, STEP = 64 * NV;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = 0; i < nt; ++i) {
    const TW* P = base + jp_off(i);
    const int64_t ld = (int64_t)(i + 1) * TB;
    const int K = i * TB;
    for (int r = wv; r < TB; r += SOLVE_NT / 64) {
      const TW* row = P + (int64_t)r * ld;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int k = lane * NV;
      for (; k + 3 * STEP < K; k += 4 * STEP) {
        const VT a0 = *(const VT*)(row + k), a1 = *(const VT*)(row + k + STEP);
        const VT a2 = *(const VT*)(row + k + 2 * STEP), a3 = *(const VT*)(row + k + 3 * STEP);
#pragma unroll
        for (int e = 0; e < NV; ++e) {
          s0 += (double)a0[e] * xs[k + e];
          s1 += (double)a1[e] * xs[k + STEP + e];
          s2 += (double)a2[e] * xs[k + 2 * STEP + e];
          s3 += (double)a3[e] * xs[k + 3 * STEP + e];
        }
      }
      for (; k < K; k += STEP) {
        const VT a0 = *(const VT*)(row + k);
#pragma unroll
        for (int e = 0; e < NV; ++e) s0 += (double)a0[e] * xs[k + e];
      }
      const double s = wave_sum((s0 + s1) + (s2 + s3));
      if (lane == 0) t[r] = v[K + r] - s;
    }
    __syncthreads();
    const TW* Li = inv + (int64_t)i * TB * TB;
    for (int r = wv; r < TB; r += SOLVE_NT / 64) {
      double s = 0.0;
      for (int c = lane; c <= r; c += 64) s += (double)Li[(int64_t)r * TB + c] * t[c];
      s = wave_sum(s);
      if (lane == 0) {
        v[K + r] = s;
        xs[K + r] = s;
      }
    }
    __syncthreads();
  }
}

// backward, right-looking: x_i = L_ii^-T v_i, then v_{<i} -= L_{i,<i}^T x_i
// (row panel i; each thread owns NV consecutive columns, rows streamed in order).
template <typename TW>
__device__ void bwd_solve(const TW* base, const TW* inv, double* v, int nt, double* xi, double* t) {
  typedef typename Vec16<TW>::type VT;
  constexpr int NV = Vec16<TW>::n;
  const int tid = threadIdx.x;
  for (int i = nt - 1; i >= 0; --i) {
    if (tid < TB) t[tid] = v[i * TB + tid];
    __syncthreads();
    if (tid < TB) {
      const TW* Li = inv + (int64_t)i * TB * TB;
      double s0 = 0.0, s1 = 0.0;
      int c = tid;
      for (; c + 1 < TB; c += 2) {
        s0 += (double)Li[(int64_t)c * TB + tid] * t[c];
        s1 += (double)Li[(int64_t)(c + 1) * TB + tid] * t[c + 1];
      }
      for (; c < TB; ++c) s0 += (double)Li[(int64_t)c * TB + tid] * t[c];
      xi[tid] = s0 + s1;
      v[i * TB + tid] = s0 + s1;
    }
    __syncthreads();
    const TW* P = base + jp_off(i);
    const int64_t ld = (int64_t)(i + 1) * TB;
    for (int col = tid * NV; col < i * TB; col += SOLVE_NT * NV) {
      double acc[NV];
#pragma unroll
      for (int e = 0; e < NV; ++e) acc[e] = 0.0;
#pragma unroll 4
      for (int r = 0; r < TB; ++r) {
        const VT a = *(const VT*)(P + (int64_t)r * ld + col);
        const double x = xi[r];
#pragma unroll
        for (int e = 0; e < NV; ++e) acc[e] += (double)a[e] * x;
      }
#pragma unroll
      for (int e = 0; e < NV; ++e) v[col + e] -= acc[e];
    }
    __syncthreads();
  }
}

template <typename TW, bool XS_LDS>
__global__ __launch_bounds__(SOLVE_NT) void k_fwd(WinVecArgs<TW> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double t[TB];
  const int m = blockIdx.x;
  const WinTab& w = a.w;
  const int T = w.T[m], tw = w.tw[m];
  const int64_t vo = w.vec[m];
  const TW* base = a.panels + w.panel[m];
  const TW* inv = a.invs + w.inv[m];
  double* xsJ = XS_LDS ? reinterpret_cast<double*>(smem_raw) : a.vJ + vo;
  fwd_solve<TW>(base, inv, a.vJ + vo, T, xsJ, t);
  if (tw > 0) {
    double* xsW = XS_LDS ? reinterpret_cast<double*>(smem_raw) : a.vW + vo;
    fwd_solve<TW>(base, inv, a.vW + vo, tw, xsW, t);
  }
}

template <typename TW>
__global__ __launch_bounds__(SOLVE_NT) void k_bwd(WinVecArgs<TW> a) {
  __shared__ double xi[TB];
  __shared__ double t[TB];
  const int m = blockIdx.x;
  const WinTab& w = a.w;
  const int T = w.T[m], tw = w.tw[m];
  const int64_t vo = w.vec[m];
  const TW* base = a.panels + w.panel[m];
  const TW* inv = a.invs + w.inv[m];
  bwd_solve<TW>(base, inv, a.vJ + vo, T, xi, t);
  if (tw > 0) bwd_solve<TW>(base, inv, a.vW + vo, tw, xi, t);
}

// L_J^-1 (c_J - K_JS g) from the stored whitened right-hand sides:
// [p; z] - [Pi; Z] g  (its W_m prefix is L_11^-1 (c_W - K_WS g)).
template <typename TW>
__global__ __launch_bounds__(256) void k_ycp(WinVecArgs<TW> a) {
  const int m = blockIdx.x;
  const WinTab& w = a.w;
  const int T = w.T[m], tw = w.tw[m];
  const int col = blockIdx.y * blockDim.x + threadIdx.x;
  if (col >= T * TB) return;
  const int64_t ld = (int64_t)T * TB;
  const TW* R = a.panels + w.rhs[m];
  double s0 = (double)R[(int64_t)a.sp * ld + col], s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int k = 0;
  for (; k + 3 < a.s; k += 4) {
    s0 -= (double)R[(int64_t)k * ld + col] * a.g[k];
    s1 -= (double)R[(int64_t)(k + 1) * ld + col] * a.g[k + 1];
    s2 -= (double)R[(int64_t)(k + 2) * ld + col] * a.g[k + 2];
    s3 -= (double)R[(int64_t)(k + 3) * ld + col] * a.g[k + 3];
  }
  for (; k < a.s; ++k) s0 -= (double)R[(int64_t)k * ld + col] * a.g[k];
  const double y = (s0 + s1) + (s2 + s3);
  const int64_t vo = w.vec[m];
  a.vJ[vo + col] = y;
  if (col < tw * TB) a.vW[vo + col] = y;
}

__device__ inline double tiled_L(const double* L, int r, int k) {
  const int ti = r / TB, tk = k / TB;
  return L[jp_off(ti) + (int64_t)(r - ti * TB) * (ti + 1) * TB + tk * TB + (k - tk * TB)];
}

// rho = L (H - L^T g), H = sum_m (hJ_m - hW_m) in block order; one workgroup
__global__ __launch_bounds__(256) void k_gres(GresArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* u = reinterpret_cast<double*>(smem_raw);  // [sp]
  const int sp = a.sp;
  for (int k = threadIdx.x; k < sp; k += blockDim.x) {
    double H = 0.0;
    for (int m = 0; m < a.M; ++m) H += a.hJ[(int64_t)m * sp + k] - a.hW[(int64_t)m * sp + k];
    double lg = 0.0;
    for (int r = k; r < sp; ++r) lg += tiled_L(a.L, r, k) * a.g[r];
    u[k] = H - lg;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < sp; r += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k <= r; ++k) s += tiled_L(a.L, r, k) * u[k];
    a.rho[r] = s;
  }
}

// g += dg, t = L^T dg; one workgroup
__global__ __launch_bounds__(256) void k_gupdate(const double* L, const double* dg, double* g, double* t, int sp) {
  for (int k = threadIdx.x; k < sp; k += blockDim.x) {
    double lg = 0.0;
    for (int r = k; r < sp; ++r) lg += tiled_L(L, r, k) * dg[r];
    t[k] = lg;
    g[k] += dg[k];
  }
}

__global__ __launch_bounds__(256) void k_vdot(const double* Vt, const double* t, double* out, int64_t n, int sp) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s = 0.0;
  for (int k = lane; k < sp; k += 64) s += Vt[i * sp + k] * t[k];
  s = wave_sum(s);
  if (lane == 0) out[i] = s;
}

__global__ __launch_bounds__(256) void k_gather(WinTab w, const double* pt, double* vJ, double* vW) {
  const int m = blockIdx.x;
  const int T = w.T[m], tw = w.tw[m];
  const int r = blockIdx.y * blockDim.x + threadIdx.x;
  if (r >= T * TB) return;
  bool v;
  const int64_t p = win_point(w, m, r, v);
  const double x = v ? pt[p] : 0.0;
  const int64_t vo = w.vec[m];
  vJ[vo + r] = x;
  if (r < tw * TB) vW[vo + r] = x;
}

__global__ __launch_bounds__(256) void k_axpy2(double* vJ, double* vW, const double* xJ, const double* xW,
                                               double alpha, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    vJ[i] += alpha * xJ[i];
    vW[i] += alpha * xW[i];
  }
}

// h = V_X x: block (m, s-tile), thread k sums over the window's rows.
__global__ __launch_bounds__(128) void k_h(HArgs a) {
  const int m = blockIdx.x, kt = blockIdx.y, k = kt * TB + threadIdx.x;
  const WinTab& w = a.w;
  const int tw = w.tw[m];
  const int64_t vo = w.vec[m];
  const int64_t wl = w.wlen[m], dl = w.dlen[m];
  const double* Vw = a.Vt + w.wstart[m] * a.sp + k;
  const double* Vd = a.Vt + w.dstart[m] * a.sp + k;
  double hj0 = 0.0, hj1 = 0.0, hw0 = 0.0, hw1 = 0.0;
  int64_t r = 0;
  for (; r + 1 < wl; r += 2) {
    const double v0 = Vw[r * a.sp], v1 = Vw[(r + 1) * a.sp];
    hj0 += v0 * a.xJ[vo + r];
    hj1 += v1 * a.xJ[vo + r + 1];
    hw0 += v0 * a.xW[vo + r];
    hw1 += v1 * a.xW[vo + r + 1];
  }
  for (; r < wl; ++r) {
    const double v0 = Vw[r * a.sp];
    hj0 += v0 * a.xJ[vo + r];
    hw0 += v0 * a.xW[vo + r];
  }
  const int64_t o = vo + (int64_t)tw * TB;
  for (r = 0; r + 1 < dl; r += 2) {
    hj0 += Vd[r * a.sp] * a.xJ[o + r];
    hj1 += Vd[(r + 1) * a.sp] * a.xJ[o + r + 1];
  }
  for (; r < dl; ++r) hj0 += Vd[r * a.sp] * a.xJ[o + r];
  a.hJ[(int64_t)m * a.sp + k] = hj0 + hj1;
  a.hW[(int64_t)m * a.sp + k] = hw0 + hw1;
}

template <typename TW>
void launch_ycp(const WinVecArgs<TW>& a, int M, int maxT, hipStream_t st) {
  hipLaunchKernelGGL(k_ycp<TW>, dim3(M, (maxT * TB + 255) / 256), dim3(256), 0, st, a);
}
template <typename TW>
void launch_fwd(const WinVecArgs<TW>& a, int M, int maxT, hipStream_t st) {
  const size_t lds = sizeof(double) * (size_t)maxT * TB;
  if (lds <= FWD_LDS_MAX)
    hipLaunchKernelGGL((k_fwd<TW, true>), dim3(M), dim3(SOLVE_NT), lds, st, a);
  else
    hipLaunchKernelGGL((k_fwd<TW, false>), dim3(M), dim3(SOLVE_NT), 0, st, a);
}
template <typename TW>
void launch_bwd(const WinVecArgs<TW>& a, int M, hipStream_t st) {
  hipLaunchKernelGGL(k_bwd<TW>, dim3(M), dim3(SOLVE_NT), 0, st, a);
}
void launch_gres(const GresArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_gres, dim3(1), dim3(256), sizeof(double) * (size_t)a.sp, st, a);
}
void launch_gupdate(const double* L, const double* dg, double* g, double* t, int sp, hipStream_t st) {
  hipLaunchKernelGGL(k_gupdate, dim3(1), dim3(256), 0, st, L, dg, g, t, sp);
}
void launch_vdot(const double* Vt, const double* t, double* out, int64_t n, int sp, hipStream_t st) {
  hipLaunchKernelGGL(k_vdot, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, Vt, t, out, n, sp);
}
void launch_gather(const WinTab& w, const double* pt, double* vJ, double* vW, int M, int maxT, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3(M, (maxT * TB + 255) / 256), dim3(256), 0, st, w, pt, vJ, vW);
}
void launch_axpy2(double* vJ, double* vW, const double* xJ, const double* xW, double alpha, int64_t nvec,
                  hipStream_t st) {
  if (nvec <= 0) return;
  const int nb = (int)std::min<int64_t>((nvec + 255) / 256, 65536);
  hipLaunchKernelGGL(k_axpy2, dim3(nb), dim3(256), 0, st, vJ, vW, xJ, xW, alpha, nvec);
}
void launch_h(const HArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_h, dim3(a.M, a.sp / TB), dim3(TB), 0, st, a);
}
hipError_t vecsolve_init() {
  for (const void* f : {(const void*)k_fwd<double, true>, (const void*)k_fwd<float, true>}) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)FWD_LDS_MAX);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template void launch_ycp<double>(const WinVecArgs<double>&, int, int, hipStream_t);
template void launch_ycp<float>(const WinVecArgs<float>&, int, int, hipStream_t);
template void launch_fwd<double>(const WinVecArgs<double>&, int, int, hipStream_t);
template void launch_fwd<float>(const WinVecArgs<float>&, int, int, hipStream_t);
template void launch_bwd<double>(const WinVecArgs<double>&, int, hipStream_t);
template void launch_bwd<float>(const WinVecArgs<float>&, int, hipStream_t);

}  // namespace lma
