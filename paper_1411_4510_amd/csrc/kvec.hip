// SE-ARD kernel-matrix times vector on 128 x 128 tiles (gfx950).
//
// One workgroup (4 wave64) per item: the item's row coordinates stay in LDS,
// each column tile is staged in LDS in turn, the cross products x_r . x_c come
// from v_mfma_f64_16x16x4f64 (wave (wr, wc) owns a 64 x 64 quadrant as 4 x 4
// sub-tiles, taken one 16-column strip at a time so that few accumulators are
// live and two workgroups fit on a CU; lane l supplies row l%16 and coordinate
// k4 + l/16 of a 4-wide step), and the epilogue forms d^2 = |x_r|^2 + |x_c|^2 - 2 x_r . x_c (all
// coordinates taken relative to the item's first row point), the
// covariance and its products with the column vectors, accumulated per row in
// registers.  Row sums are reduced in a fixed order (lane shuffles, then the
// two column halves), so results do not depend on scheduling.
#include "engine.h"
#include "kvec.h"
#include "mfma_core.h"
#include "misc.h"

namespace lma {

__device__ inline double vdot_wave(const double* __restrict__ a, const double* __restrict__ b, int n, int lane) {
  double s0 = 0.0, s1 = 0.0;
  int k = lane;
  for (; k + 64 < n; k += 128) {
    s0 += a[k] * b[k];
    s1 += a[k + 64] * b[k + 64];
  }
  for (; k < n; k += 64) s0 += a[k] * b[k];
  double s = s0 + s1;
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  return s;
}

__global__ __launch_bounds__(256) void k_kvec(KvArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int d = a.d, dp = (d + 3) & ~3, ldx = dp + 1;
  double* xr = reinterpret_cast<double*>(smem_raw);  // [TB][ldx] row coordinates
  double* xc = xr + TB * ldx;                        // [TB][ldx] column coordinates
  double* nrm_r = xc + TB * ldx;                     // [TB]
  double* nrm_c = nrm_r + TB;                        // [TB]
  double* cv0 = nrm_c + TB;                          // [TB]
  double* cv1 = cv0 + TB;                            // [TB]
  double* red = cv1 + TB;                            // [2 sums][2 column halves][TB]
  double* vd = red + 4 * TB;                         // [2][TB] whitened-row dots
  const int logical = xcd_logical(blockIdx.x, gridDim.x);
  if (logical >= a.nitems) return;
  const KvItem it = a.items[logical];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;

  // coordinates relative to the item's first row point (distances are
  // translation invariant; small norms keep |x|^2 + |y|^2 - 2 x.y accurate)
  __shared__ double org[MAX_D];
  if (tid < d) org[tid] = it.nr > 0 ? it.x[tid] : 0.0;
  __syncthreads();
  for (int idx = tid; idx < TB * dp; idx += NT) {
    const int r = idx / dp, k = idx - r * dp;
    xr[r * ldx + k] = (r < it.nr && k < d) ? it.x[(int64_t)r * d + k] - org[k] : 0.0;
  }
  __syncthreads();
  if (tid < TB) {
    double s = 0.0;
    for (int k = 0; k < dp; ++k) s += xr[tid * ldx + k] * xr[tid * ldx + k];
    nrm_r[tid] = s;
  }
  double s0[4][4], s1[4][4];
#pragma unroll
  for (int ra = 0; ra < 4; ++ra)
#pragma unroll
    for (int v = 0; v < 4; ++v) s0[ra][v] = s1[ra][v] = 0.0;
  const double sf2 = a.sf2;

  for (int c = it.c0; c < it.c1; ++c) {
    const KvCol col = a.cols[c];
    __syncthreads();  // the previous column tile is consumed
    for (int r = tid >> 1; r < TB; r += NT / 2)
      for (int k = tid & 1; k < dp; k += 2)
        xc[r * ldx + k] = (r < col.nc && k < d) ? col.x[(int64_t)r * d + k] - org[k] : 0.0;
    if (tid < TB) {
      cv0[tid] = (col.v0 && tid < col.nc) ? col.v0[tid] : 0.0;
      cv1[tid] = (col.v1 && tid < col.nc) ? col.v1[tid] : 0.0;
    }
    __syncthreads();
    if (tid < TB) {
      double s = 0.0;
      for (int k = 0; k < dp; ++k) s += xc[tid * ldx + k] * xc[tid * ldx + k];
      nrm_c[tid] = s;
    }
    __syncthreads();  // column norms written
    // one 16-column strip at a time: its 4 product tiles, then their covariance
    // entries (keeps 16 accumulators live instead of 64)
#pragma unroll 1
    for (int rb = 0; rb < 4; ++rb) {
      dv4 acc[4];
#pragma unroll
      for (int ra = 0; ra < 4; ++ra) acc[ra] = Mfma<double>::op(0.0, 0.0, dv4{0.0, 0.0, 0.0, 0.0});
      const int cb = (wc * 64 + rb * 16 + (lane & 15)) * ldx + (lane >> 4);
      for (int k4 = 0; k4 < dp; k4 += 4) {
        const double bf = xc[cb + k4];
#pragma unroll
        for (int ra = 0; ra < 4; ++ra) {
          const double af = xr[(wr * 64 + ra * 16 + (lane & 15)) * ldx + k4 + (lane >> 4)];
          acc[ra] = Mfma<double>::op(af, bf, acc[ra]);
        }
      }
      const int cc = wc * 64 + rb * 16 + (lane & 15);
      const double nc = nrm_c[cc], v0 = cv0[cc], v1 = cv1[cc];
#pragma unroll
      for (int ra = 0; ra < 4; ++ra)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = wr * 64 + ra * 16 + Mfma<double>::row(lane, v);
          double d2 = nrm_r[rr] + nc - 2.0 * acc[ra][v];
          d2 = d2 > 0.0 ? d2 : 0.0;
          const double kv = sf2 * exp(-0.5 * d2);
          s0[ra][v] += kv * v0;
          s1[ra][v] += kv * v1;
        }
    }
  }

  // row sums: over the 16 column lanes, then over the two column halves
#pragma unroll
  for (int ra = 0; ra < 4; ++ra)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double x0 = s0[ra][v], x1 = s1[ra][v];
      for (int o = 1; o < 16; o <<= 1) {
        x0 += __shfl_xor(x0, o);
        x1 += __shfl_xor(x1, o);
      }
      if ((lane & 15) == 0) {
        const int rr = wr * 64 + ra * 16 + Mfma<double>::row(lane, v);
        red[(0 * 2 + wc) * TB + rr] = x0;
        red[(1 * 2 + wc) * TB + rr] = x1;
      }
    }
  // whitened-row dots (one wave per row)
  for (int r = w; r < TB; r += NT / 64) {
    double d0 = 0.0, d1 = 0.0;
    if (it.vt != nullptr && r < it.nr) {
      const double* vr = it.vt + (int64_t)r * a.sp;
      if (it.h0) d0 = vdot_wave(vr, it.h0, a.sp, lane);
      if (it.h1 && it.flag) d1 = vdot_wave(vr, it.h1, a.sp, lane);
    }
    if (lane == 0) {
      vd[r] = d0;
      vd[TB + r] = d1;
    }
  }
  __syncthreads();
  if (tid < TB) {
    const int r = tid;
    const double acc0 = red[0 * TB + r] + red[1 * TB + r];
    const double acc1 = red[2 * TB + r] + red[3 * TB + r];
    if (a.mode == KV_CG) {
      if (r < it.nr) it.out0[r] = it.base0[r] - acc0;
    } else if (a.mode == KV_MEAN) {
      if (r < it.nr) it.out0[r] = a.mu + acc0 - acc1 - vd[r];
    } else {
      if (r < it.nr) {
        it.out0[r] = it.base0[r] - (acc0 + a.sn2 * it.self0[r] - vd[r]);
        if (it.flag) it.out1[r] = it.base0[r] - (acc1 + a.sn2 * it.self1[r] - vd[TB + r]);
      } else {
        it.out0[r] = 0.0;
        if (it.flag) it.out1[r] = 0.0;
      }
    }
  }
}

__global__ void k_hq(const double* __restrict__ hJ, const double* __restrict__ hW, double* __restrict__ hq, int M,
                     int B, int sp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)M * sp) return;
  const int q = (int)(e / sp), k = (int)(e - (int64_t)q * sp);
  double s = 0.0;
  for (int dl = 0; dl <= B && dl <= q; ++dl) {
    s += hJ[(int64_t)(q - dl) * sp + k];
    if (dl > 0) s -= hW[(int64_t)(q - dl) * sp + k];
  }
  hq[e] = s;
}

static size_t kvec_lds(int d) {
  const int ldx = ((d + 3) & ~3) + 1;
  return sizeof(double) * (size_t)(2 * TB * ldx + 10 * TB);
}

void launch_kvec(const KvArgs& a, hipStream_t st) {
  if (a.nitems <= 0) return;
  const int nb = ((a.nitems + 7) / 8) * 8;
  hipLaunchKernelGGL(k_kvec, dim3(nb), dim3(NT), kvec_lds(a.d), st, a);
}

void launch_hq(const double* hJ, const double* hW, double* hq, int M, int B, int sp, hipStream_t st) {
  const int64_t n = (int64_t)M * sp;
  hipLaunchKernelGGL(k_hq, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, hJ, hW, hq, M, B, sp);
}

hipError_t kvec_init() {
  return hipFuncSetAttribute((const void*)k_kvec, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kvec_lds(MAX_D));
}

}  // namespace lma
