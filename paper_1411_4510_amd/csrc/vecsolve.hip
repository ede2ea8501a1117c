// Vector solves with the stored window factors and the predictive mean.
//
// With g = Sigma_ddot_SS^-1 y_ddot_S and beta_X = R_X^-1 (c_X - K_XS g) for the
// windows X = J_m and the separators X = W_m, the predictive mean of Eq. (3)
// for u in test block q is
//   mu + k_u^T g + sum_{m=q-B..q} R_{u,J_m} beta_{J_m} - sum_{m=q-B..q-1} R_{u,W_m} beta_{W_m}.
// (Woodbury on Sigma_bar_DD = Q + R_bar and the signed window sum of
// R_bar_DD^-1 that the banded factor of Lemma 1 gives; the separator term of
// window q cancels against its own leading block.)  Only vector solves are
// needed, so they run in float64 arithmetic even on float32 factors.
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

// forward: v <- L^-1 v over the first nt column tiles
template <typename TW>
__device__ void fwd_solve(const TW* base, const TW* inv, double* v, int nt, double* tmp) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = 0; i < nt; ++i) {
    const TW* P = base + jp_off(i);
    const int64_t ld = (int64_t)(i + 1) * TB;
    for (int q = 0; q < TB / 4; ++q) {
      const int r = wv + 4 * q;
      double s = 0.0;
      for (int k = lane; k < i * TB; k += 64) s += (double)P[(int64_t)r * ld + k] * v[k];
      s = wave_sum(s);
      if (lane == 0) tmp[r] = v[i * TB + r] - s;
    }
    __syncthreads();
    if (tid < TB) {
      const TW* Li = inv + (int64_t)i * TB * TB + (int64_t)tid * TB;
      double s = 0.0;
      for (int c = 0; c <= tid; ++c) s += (double)Li[c] * tmp[c];
      v[i * TB + tid] = s;
    }
    __syncthreads();
  }
}

// backward: v <- L^-T v over the first nt column tiles
template <typename TW>
__device__ void bwd_solve(const TW* base, const TW* inv, double* v, int nt, double* tmp, double* part) {
  const int tid = threadIdx.x, r = tid & (TB - 1), h = tid >> 7;
  for (int i = nt - 1; i >= 0; --i) {
    double s = 0.0;
    for (int k = i + 1 + h; k < nt; k += 2) {
      const TW* P = base + jp_off(k) + (int64_t)i * TB;
      const int64_t ld = (int64_t)(k + 1) * TB;
      const double* vk = v + (int64_t)k * TB;
      for (int c = 0; c < TB; ++c) s += (double)P[(int64_t)c * ld + r] * vk[c];
    }
    part[h * TB + r] = s;
    __syncthreads();
    if (tid < TB) tmp[tid] = v[i * TB + tid] - part[tid] - part[TB + tid];
    __syncthreads();
    if (tid < TB) {
      const TW* Li = inv + (int64_t)i * TB * TB;
      double acc = 0.0;
      for (int c = tid; c < TB; ++c) acc += (double)Li[(int64_t)c * TB + tid] * tmp[c];
      v[i * TB + tid] = acc;
    }
    __syncthreads();
  }
}

template <typename TW>
__global__ __launch_bounds__(256) void k_vec_solve(VecSolveArgs<TW> a) {
  __shared__ double tmp[TB];
  __shared__ double part[2 * TB];
  const int m = blockIdx.x, tid = threadIdx.x;
  const WinTab& w = a.w;
  const int T = w.T[m], tw = w.tw[m];
  const int64_t vo = w.vec[m];
  const TW* base = a.panels + w.panel[m];
  const TW* inv = a.invs + w.inv[m];
  double* tJ = a.tJ + vo;
  double* tW = a.tW + vo;
  for (int r = tid; r < T * TB; r += blockDim.x) {
    bool valid;
    const int64_t pt = win_point(w, m, r, valid);
    tJ[r] = valid ? (a.rhs_pt ? a.rhs_pt[pt] : a.rhsJ[vo + r]) : 0.0;
    if (r < tw * TB) tW[r] = valid ? (a.rhs_pt ? a.rhs_pt[pt] : a.rhsW[vo + r]) : 0.0;
  }
  __syncthreads();
  fwd_solve<TW>(base, inv, tJ, T, tmp);
  bwd_solve<TW>(base, inv, tJ, T, tmp, part);
  if (tw > 0) {
    fwd_solve<TW>(base, inv, tW, tw, tmp);
    bwd_solve<TW>(base, inv, tW, tw, tmp, part);
  }
  for (int r = tid; r < T * TB; r += blockDim.x) {
    const double xj = tJ[r], xw = r < tw * TB ? tW[r] : 0.0;
    a.xJ[vo + r] = a.accumulate ? a.xJ[vo + r] + xj : xj;
    a.xW[vo + r] = a.accumulate ? a.xW[vo + r] + xw : xw;
  }
}

// h = V_X x: block (m, s-tile), thread k sums over the window's rows.
__global__ __launch_bounds__(128) void k_h(HArgs a) {
  const int m = blockIdx.x, kt = blockIdx.y, k = kt * TB + threadIdx.x;
  const WinTab& w = a.w;
  const int T = w.T[m], tw = w.tw[m];
  const int64_t vo = w.vec[m];
  double hj = 0.0, hw = 0.0;
  for (int r = 0; r < T * TB; ++r) {
    bool valid;
    const int64_t pt = win_point(w, m, r, valid);
    if (!valid) continue;
    const double v = a.Vt[pt * a.sp + k];
    hj += v * a.xJ[vo + r];
    if (r < tw * TB) hw += v * a.xW[vo + r];
  }
  a.hJ[(int64_t)m * a.sp + k] = hj;
  a.hW[(int64_t)m * a.sp + k] = hw;
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
void launch_vec_solve(const VecSolveArgs<TW>& a, int M, hipStream_t st) {
  hipLaunchKernelGGL(k_vec_solve<TW>, dim3(M), dim3(256), 0, st, a);
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
template void launch_vec_solve<double>(const VecSolveArgs<double>&, int, hipStream_t);
template void launch_vec_solve<float>(const VecSolveArgs<float>&, int, hipStream_t);

}  // namespace lma
