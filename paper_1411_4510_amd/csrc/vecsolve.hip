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
// triangular solves of one vector per window (one workgroup per window)
// ---------------------------------------------------------------------------

// forward, left-looking: t_i = v_i - L_{i,<i} v_{<i}, v_i = L_ii^-1 t_i.
// One wave per row for the panel dot (lanes along k, coalesced).
template <typename TW>
__device__ void fwd_solve(const TW* base, const TW* inv, double* v, int nt, double* t) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = 0; i < nt; ++i) {
    const TW* P = base + jp_off(i);
    const int64_t ld = (int64_t)(i + 1) * TB;
    const int K = i * TB;
    for (int q = 0; q < TB / 4; ++q) {
      const int r = wv + 4 * q;
      const TW* row = P + (int64_t)r * ld;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int k = lane;
      for (; k + 192 < K; k += 256) {
        s0 += (double)row[k] * v[k];
        s1 += (double)row[k + 64] * v[k + 64];
        s2 += (double)row[k + 128] * v[k + 128];
        s3 += (double)row[k + 192] * v[k + 192];
      }
      for (; k < K; k += 64) s0 += (double)row[k] * v[k];
      const double s = wave_sum((s0 + s1) + (s2 + s3));
      if (lane == 0) t[r] = v[K + r] - s;
    }
    __syncthreads();
    const TW* Li = inv + (int64_t)i * TB * TB;
    for (int q = 0; q < TB / 4; ++q) {
      const int r = wv + 4 * q;
      double s = 0.0;
      for (int c = lane; c <= r; c += 64) s += (double)Li[(int64_t)r * TB + c] * t[c];
      s = wave_sum(s);
      if (lane == 0) v[K + r] = s;
    }
    __syncthreads();
  }
}

// backward, right-looking: x_i = L_ii^-T v_i, then v_{<i} -= L_{i,<i}^T x_i
// (row panel i, one thread per column, coalesced along the row).
template <typename TW>
__device__ void bwd_solve(const TW* base, const TW* inv, double* v, int nt, double* xi, double* t) {
  const int tid = threadIdx.x;
  for (int i = nt - 1; i >= 0; --i) {
    if (tid < TB) t[tid] = v[i * TB + tid];
    __syncthreads();
    if (tid < TB) {
      const TW* Li = inv + (int64_t)i * TB * TB;
      double s = 0.0;
      for (int c = tid; c < TB; ++c) s += (double)Li[(int64_t)c * TB + tid] * t[c];
      xi[tid] = s;
      v[i * TB + tid] = s;
    }
    __syncthreads();
    const TW* P = base + jp_off(i);
    const int64_t ld = (int64_t)(i + 1) * TB;
    for (int col = tid; col < i * TB; col += blockDim.x) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 4
      for (int r = 0; r < TB; r += 4) {
        s0 += (double)P[(int64_t)r * ld + col] * xi[r];
        s1 += (double)P[(int64_t)(r + 1) * ld + col] * xi[r + 1];
        s2 += (double)P[(int64_t)(r + 2) * ld + col] * xi[r + 2];
        s3 += (double)P[(int64_t)(r + 3) * ld + col] * xi[r + 3];
      }
      v[col] -= (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
  }
}

template <typename TW>
__global__ __launch_bounds__(256) void k_fwd(WinVecArgs<TW> a) {
  __shared__ double t[TB];
  const int m = blockIdx.x;
  const WinTab& w = a.w;
  const int T = w.T[m], tw = w.tw[m];
  const int64_t vo = w.vec[m];
  const TW* base = a.panels + w.panel[m];
  const TW* inv = a.invs + w.inv[m];
  fwd_solve<TW>(base, inv, a.vJ + vo, T, t);
  if (tw > 0) fwd_solve<TW>(base, inv, a.vW + vo, tw, t);
}

template <typename TW>
__global__ __launch_bounds__(256) void k_bwd(WinVecArgs<TW> a) {
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

// r = c' - R_X x in float64 for the rows of tile i of window m (X = J_m, and
// X = W_m when i < tw); the covariance is recomputed from the coordinates.
__global__ __launch_bounds__(256) void k_kmv(KmvArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int d = a.d;
  double* xr = reinterpret_cast<double*>(smem_raw);  // [d][TB]
  double* xc = xr + d * TB;                          // [d][TB]
  double* xvJ = xc + d * TB;                         // [TB]
  double* xvW = xvJ + TB;                            // [TB]
  double* part = xvW + TB;                           // [4][TB]
  const int m = blockIdx.x, i = blockIdx.y, tid = threadIdx.x;
  const WinTab& w = a.w;
  const int T = w.T[m], tw = w.tw[m];
  if (i >= T) return;
  const int64_t vo = w.vec[m];
  const int r = tid & (TB - 1), h = tid >> 7;
  for (int idx = tid; idx < TB * d; idx += blockDim.x) {
    const int rr = idx / d, tt = idx - rr * d;
    bool v;
    const int64_t p = win_point(w, m, i * TB + rr, v);
    xr[tt * TB + rr] = v ? a.Xs[p * d + tt] : 0.0;
  }
  bool va;
  const int64_t pa = win_point(w, m, i * TB + r, va);
  double sj = 0.0, sw = 0.0;
  for (int j = 0; j < T; ++j) {
    __syncthreads();
    for (int idx = tid; idx < TB * d; idx += blockDim.x) {
      const int cc = idx / d, tt = idx - cc * d;
      bool v;
      const int64_t p = win_point(w, m, j * TB + cc, v);
      xc[tt * TB + cc] = v ? a.Xs[p * d + tt] : 0.0;
    }
    if (tid < TB) {
      bool v;
      win_point(w, m, j * TB + tid, v);
      xvJ[tid] = v ? a.xJ[vo + j * TB + tid] : 0.0;
      xvW[tid] = (v && j < tw) ? a.xW[vo + j * TB + tid] : 0.0;
    }
    __syncthreads();
    if (va) {
      const bool dow = i < tw && j < tw;
      for (int c = h; c < TB; c += 2) {
        const double xj = xvJ[c], xw = xvW[c];
        if (xj == 0.0 && xw == 0.0) continue;
        double s = 0.0;
        for (int t = 0; t < d; ++t) {
          const double df = xr[t * TB + r] - xc[t * TB + c];
          s += df * df;
        }
        const double kv = a.sf2 * exp(-0.5 * s);
        sj += kv * xj;
        if (dow) sw += kv * xw;
      }
    }
  }
  part[h * TB + r] = sj;
  part[(2 + h) * TB + r] = sw;
  __syncthreads();
  if (tid < TB) {
    const int row = i * TB + r;
    double resJ = 0.0, resW = 0.0;
    if (va) {
      const double* vt = a.Vt + pa * a.sp;
      const double* hj = a.hJ + (int64_t)m * a.sp;
      const double* hw = a.hW + (int64_t)m * a.sp;
      double qj = 0.0, qw = 0.0;
      for (int k = 0; k < a.sp; ++k) {
        qj += vt[k] * hj[k];
        qw += vt[k] * hw[k];
      }
      const double rhs = a.rhs_pt[pa];
      resJ = rhs - (part[r] + part[TB + r] + a.sn2 * a.xJ[vo + row] - qj);
      if (i < tw) resW = rhs - (part[2 * TB + r] + part[3 * TB + r] + a.sn2 * a.xW[vo + row] - qw);
    }
    a.rJ[vo + row] = resJ;
    if (i < tw) a.rW[vo + row] = resW;
  }
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

// c' = c - K_DS g, one wave per training point.
__global__ __launch_bounds__(256) void k_cg(CgArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= a.n) return;
  const double* xi = a.Xs + i * a.d;
  double s = 0.0;
  for (int k = lane; k < a.s; k += 64) s += a.sf2 * exp(-0.5 * sqd(xi, a.Ss + (int64_t)k * a.d, a.d)) * a.g[k];
  s = wave_sum(s);
  if (lane == 0) a.out[i] = a.c[i] - s;
}

// predictive mean, one wave per test point
__global__ __launch_bounds__(256) void k_mean(MeanArgs a) {
  __shared__ double xu_s[4][MAX_D];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t u = (int64_t)blockIdx.x * 4 + wv;
  const bool live = u < a.n_u;
  if (live)
    for (int t = lane; t < a.d; t += 64) xu_s[wv][t] = a.Us[u * a.d + t];
  __syncthreads();
  if (!live) return;
  const double* xu = xu_s[wv];
  const WinTab& w = a.w;
  double acc = 0.0;
  for (int k = lane; k < a.s; k += 64) acc += a.sf2 * exp(-0.5 * sqd(xu, a.Ss + (int64_t)k * a.d, a.d)) * a.g[k];
  const int q = a.ublk[u];
  const double* vu = a.VtU + u * a.sp;
  for (int dl = 0; dl <= a.B && dl <= q; ++dl) {
    const int m = q - dl;
    const int T = w.T[m], tw = w.tw[m];
    const int64_t vo = w.vec[m];
    for (int r = lane; r < T * TB; r += 64) {
      bool valid;
      const int64_t pt = win_point(w, m, r, valid);
      if (!valid) continue;
      const double kv = a.sf2 * exp(-0.5 * sqd(xu, a.Xs + pt * a.d, a.d));
      acc += kv * a.xJ[vo + r];
      if (dl > 0 && r < tw * TB) acc -= kv * a.xW[vo + r];
    }
    const double* hj = a.hJ + (int64_t)m * a.sp;
    const double* hw = a.hW + (int64_t)m * a.sp;
    for (int k = lane; k < a.sp; k += 64) {
      acc -= vu[k] * hj[k];
      if (dl > 0) acc += vu[k] * hw[k];
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) a.mean[u] = a.mu + acc;
}

template <typename TW>
void launch_ycp(const WinVecArgs<TW>& a, int M, int maxT, hipStream_t st) {
  hipLaunchKernelGGL(k_ycp<TW>, dim3(M, (maxT * TB + 255) / 256), dim3(256), 0, st, a);
}
template <typename TW>
void launch_fwd(const WinVecArgs<TW>& a, int M, hipStream_t st) {
  hipLaunchKernelGGL(k_fwd<TW>, dim3(M), dim3(256), 0, st, a);
}
template <typename TW>
void launch_bwd(const WinVecArgs<TW>& a, int M, hipStream_t st) {
  hipLaunchKernelGGL(k_bwd<TW>, dim3(M), dim3(256), 0, st, a);
}
void launch_kmv(const KmvArgs& a, int M, int maxT, hipStream_t st) {
  const size_t lds = sizeof(double) * (size_t)(2 * a.d * TB + 6 * TB);
  hipLaunchKernelGGL(k_kmv, dim3(M, maxT), dim3(256), lds, st, a);
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
  const int nb = (int)std::min<int64_t>((nvec + 255) / 256, 65536);
  hipLaunchKernelGGL(k_axpy2, dim3(nb), dim3(256), 0, st, vJ, vW, xJ, xW, alpha, nvec);
}
void launch_h(const HArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_h, dim3(a.M, a.sp / TB), dim3(TB), 0, st, a);
}
void launch_cg(const CgArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_cg, dim3((unsigned)((a.n + 3) / 4)), dim3(256), 0, st, a);
}
void launch_mean(const MeanArgs& a, hipStream_t st) {
  if (a.n_u <= 0) return;
  hipLaunchKernelGGL(k_mean, dim3((unsigned)((a.n_u + 3) / 4)), dim3(256), 0, st, a);
}
hipError_t vecsolve_init() {
  return hipFuncSetAttribute((const void*)k_kmv, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(double) * (2 * MAX_D * TB + 6 * TB)));
}

template void launch_ycp<double>(const WinVecArgs<double>&, int, int, hipStream_t);
template void launch_ycp<float>(const WinVecArgs<float>&, int, int, hipStream_t);
template void launch_fwd<double>(const WinVecArgs<double>&, int, hipStream_t);
template void launch_fwd<float>(const WinVecArgs<float>&, int, hipStream_t);
template void launch_bwd<double>(const WinVecArgs<double>&, int, hipStream_t);
template void launch_bwd<float>(const WinVecArgs<float>&, int, hipStream_t);

}  // namespace lma
