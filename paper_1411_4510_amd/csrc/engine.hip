// Device kernels of the tiled Cholesky / triangular-solve engine (gfx950).
// The MFMA tile core (operand layout, prefetch pipeline) is in mfma_core.h.
#include "engine.h"
#include "mfma_core.h"

#include <type_traits>

namespace lma {

// ---------------------------------------------------------------------------
// update: C_ij = K_ij - V_i V_j^T - sum_{k<j} L_ik L_jk^T for every item (p, i)
// ---------------------------------------------------------------------------
template <typename T, bool MIXED>
__global__ __launch_bounds__(NT) void k_update(StepArgs<T> a) {
  // covariance tile and V-part precision: float64 when T is double or MIXED
  typedef typename std::conditional<MIXED, double, T>::type TK;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int logical = xcd_logical(blockIdx.x, gridDim.x);
  if (logical >= a.nitems) return;
  const WorkItem it = a.items[logical];
  const ProbDesc pd = a.pd[it.p];
  const RowTile<T> ri = a.rt[pd.first + it.tile];
  const RowTile<T> rj = a.rt[pd.first + a.j];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;

  typename Mfma<TK>::acc accv[4][4];   // V_i V_j^T
  typename Mfma<T>::acc accl[4][4];    // sum_k L_ik L_jk^T (aliases accv when not MIXED)
  const bool band = ri.src == SRC_BAND;    // V part already inside the band entries
  const bool tband = ri.src == SRC_TBAND;  // likewise for test rows
  if (band || tband) {
    // Band rows start from minus their residual entries, so that the band reads
    // are in flight with the first operand loads instead of after the k loop;
    // the epilogue then stores -(accumulator).  Every lane issues its 64 reads
    // unconditionally (padding rows and columns read a valid entry of the tile and
    // are masked to zero), and the accumulators are started through an MFMA, as
    // in zero_acc, so that they stay in their register file.
    const int nvr = ri.nvalid, nvc = rj.nvalid;
    int64_t rowp[4][4], rowb[4][4], colq[4], colb[4];
#pragma unroll
    for (int cs = 0; cs < 4; ++cs) {
      const int col = wc * 64 + cs * 16 + (lane & 15);
      colq[cs] = rj.pt0 + (col < nvc ? col : nvc - 1);
      colb[cs] = tband ? 0 : a.brow[colq[cs]];
    }
#pragma unroll
    for (int rs = 0; rs < 4; ++rs)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 64 + rs * 16 + Mfma<TK>::row(lane, v);
        rowp[rs][v] = ri.pt0 + (row < nvr ? row : nvr - 1);
        rowb[rs][v] = a.brow[rowp[rs][v]];
      }
#pragma unroll
    for (int rs = 0; rs < 4; ++rs)
#pragma unroll
      for (int cs = 0; cs < 4; ++cs) {
        typename Mfma<TK>::acc r0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = wr * 64 + rs * 16 + Mfma<TK>::row(lane, v);
          const int col = wc * 64 + cs * 16 + (lane & 15);
          const int64_t p = rowp[rs][v], q = colq[cs];
          const int64_t e = (tband || q <= p) ? rowb[rs][v] + q : colb[cs] + p;
          const TK kv = (TK)a.band[e];
          r0[v] = (row < nvr && col < nvc) ? -kv : TK(0);
        }
        accv[rs][cs] = Mfma<TK>::op(TK(0), TK(0), r0);
      }
  } else {
    zero_acc<TK>(accv);
  }
  if constexpr (MIXED) zero_acc<T>(accl);
  const TK* vi = MIXED ? (const TK*)ri.vt64 : (const TK*)ri.vt;
  const TK* vj = MIXED ? (const TK*)rj.vt64 : (const TK*)rj.vt;
  if (!band && !tband && vi != nullptr && vj != nullptr && a.vlen > 0)
    wave_gemm<TK, TK>(accv, vi, a.vld, ri.nvalid, vj, a.vld, rj.nvalid, 0, a.vlen, wr * 64, wc * 64, lane);
  // factor columns kb .. j-1 (a row is zero left of its kbeg)
  const int kb = ri.kbeg > rj.kbeg ? ri.kbeg : rj.kbeg;
  if (a.j > kb) {
    const T* pa = ri.panel + (int64_t)(kb - ri.kbeg) * TB;
    const T* pb = rj.panel + (int64_t)(kb - rj.kbeg) * TB;
    if constexpr (MIXED)  // float32 products, sums folded into the float64 accumulators
      wave_gemm_fold(accl, pa, ri.ld, ri.nstore, pb, rj.ld, rj.nstore, 0, (a.j - kb) * TB, wr * 64, wc * 64, lane,
                     accv);
    else
      wave_gemm<T, T>(accv, pa, ri.ld, ri.nstore, pb, rj.ld, rj.nstore, 0, (a.j - kb) * TB, wr * 64, wc * 64, lane);
  }

  const int d = a.d;
  TK* xr = reinterpret_cast<TK*>(smem_raw);  // [d][TB] row-side coordinates
  TK* xc = xr + d * TB;                      // [d][TB] column-side coordinates
  const bool kern = ri.src == SRC_KERNEL;
  if (kern) {
    const TK* xsi = MIXED ? (const TK*)ri.xs64 : (const TK*)ri.xs;
    const TK* xsj = MIXED ? (const TK*)rj.xs64 : (const TK*)rj.xs;
    for (int idx = tid; idx < TB * d; idx += NT) {
      const int r = idx / d, t = idx - r * d;
      xr[t * TB + r] = r < ri.nvalid ? xsi[(int64_t)r * d + t] : TK(0);
      xc[t * TB + r] = r < rj.nvalid ? xsj[(int64_t)r * d + t] : TK(0);
    }
  }
  __syncthreads();
  const bool diag = ri.is_j && (it.tile == a.j);
  const TK sf2 = (TK)a.sf2, sn2 = (TK)a.sn2;
  T* out = ri.panel + (int64_t)(a.j - ri.kbeg) * TB;
  const bool ident = ri.src == SRC_IDENT;
  const bool ident_here = ident && ri.kbeg == a.j;
  // squared distances of the lane's 64 entries, one coordinate at a time
  TK sq[4][4][4];
#pragma unroll
  for (int rs = 0; rs < 4; ++rs)
#pragma unroll
    for (int cs = 0; cs < 4; ++cs)
#pragma unroll
      for (int v = 0; v < 4; ++v) sq[rs][cs][v] = TK(0);
  if (kern) {
    for (int t = 0; t < d; ++t) {
      TK cv[4];
#pragma unroll
      for (int cs = 0; cs < 4; ++cs) cv[cs] = xc[t * TB + wc * 64 + cs * 16 + (lane & 15)];
#pragma unroll
      for (int rs = 0; rs < 4; ++rs)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const TK rv = xr[t * TB + wr * 64 + rs * 16 + Mfma<TK>::row(lane, v)];
#pragma unroll
          for (int cs = 0; cs < 4; ++cs) {
            const TK df = rv - cv[cs];
            sq[rs][cs][v] += df * df;
          }
        }
    }
  }
#pragma unroll
  for (int rs = 0; rs < 4; ++rs) {
#pragma unroll
    for (int cs = 0; cs < 4; ++cs) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 64 + rs * 16 + Mfma<TK>::row(lane, v);
        const int col = wc * 64 + cs * 16 + (lane & 15);
        TK kv = TK(0);
        if (ident) {
          kv = (ident_here && row == col) ? TK(1) : TK(0);  // exact at padding too
        } else if (row < ri.nvalid && col < rj.nvalid) {
          if (kern) {
            kv = sf2 * k_exp(TK(-0.5) * sq[rs][cs][v]);
            if (diag && row == col) kv += sn2;
          } else if (band || tband) {
            kv = TK(0);  // the residual entry started the accumulator (negated)
          } else if (ri.src == SRC_EXPLICIT) {
            kv = (TK)ri.expl[(int64_t)row * ri.eld + (int64_t)a.j * TB + col];
          } else {
            kv = row == 0 ? (TK)rj.cv[col] : TK(0);
          }
        } else if (diag && row == col) {
          kv = TK(1);
        }
        T val;
        if (row >= ri.nvalid || col >= rj.nvalid)
          val = (T)kv;  // padding: identity on the diagonal tile, zero elsewhere
        else if constexpr (MIXED)
          val = (T)(kv - accv[rs][cs][v]);  // accl was folded into accv
        else
          val = (T)(kv - accv[rs][cs][v]);
        if (row < ri.nstore) out[(int64_t)row * ri.ld + col] = val;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// diag: Cholesky of the diagonal tile (j, j) in LDS, its log-diagonal, and the
// inverse of the factor for the triangular solves of the tiles below.
// ---------------------------------------------------------------------------
// The tile is factored and inverted in float64 for every storage type (the
// float32 window factors of the mixed mode included): the diagonal tiles of
// late column steps hold Schur complements near the noise level, and their
// factor and inverse feed every later tile.
//
// Both run on 32 x 32 blocks.  Factor, for each block column kb: one wave
// factors the diagonal block in lock step (no workgroup barrier per column),
// the rows below are solved against it one row per thread, and the trailing
// block update is spread over the workgroup.  Inverse (in place, X = L^-1):
// the four diagonal blocks are inverted by the four waves at once, then block
// columns right to left: T_ib = sum_{k=jb+1..ib} X_ib,k L_k,jb for every block
// row ib below jb, and X_ib,jb = -T_ib X_jb,jb.  About twenty workgroup
// barriers per tile instead of two per column.
constexpr int DB = 32;          // block size of the diagonal-tile algorithms
constexpr int DNB = TB / DB;    // blocks per tile side
constexpr int DT_LD = DB + 1;   // row stride of the block products' scratch

__device__ inline void wave_sync_lds() {
  // LDS writes of this wave are visible to its other lanes after this point
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__global__ __launch_bounds__(NT) void k_diag(StepArgs<T> a, const int32_t* __restrict__ plist) {
  typedef double TA;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TA* A = reinterpret_cast<TA*>(smem_raw);  // [TB][DIAG_LD]
  TA* Tt = A + TB * DIAG_LD;                // [DNB-1][DB][DT_LD] block products
  __shared__ int bad;
  __shared__ double lsum[NT / 64];
  const int p = plist[blockIdx.x];
  const ProbDesc pd = a.pd[p];
  const RowTile<T> rj = a.rt[pd.first + a.j];
  T* src = rj.panel + (int64_t)a.j * TB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) bad = 0;
  for (int idx = tid; idx < TB * TB; idx += NT) {
    const int r = idx >> 7, c = idx & (TB - 1);
    A[r * DIAG_LD + c] = c <= r ? (TA)src[(int64_t)r * rj.ld + c] : TA(0);
  }
  __syncthreads();

  // ---- factor
  for (int kb = 0; kb < DNB; ++kb) {
    const int b0 = kb * DB;
    if (w == 0) {  // diagonal block, right-looking, one wave in lock step
      const int rl = lane & 31, h = lane >> 5, r = b0 + rl;
      for (int k = 0; k < DB; ++k) {
        const int kk = b0 + k;
        TA dkk = A[kk * DIAG_LD + kk];
        const bool ok = dkk > TA(0);
        if (!ok) dkk = TA(1);
        const TA piv = k_sqrt(dkk), ip = TA(1) / piv;
        wave_sync_lds();  // every lane has read the pivot
        if (h == 0) {
          if (rl > k) {
            A[r * DIAG_LD + kk] *= ip;
          } else if (rl == k) {
            A[kk * DIAG_LD + kk] = piv;
            if (!ok) bad = 1;
          }
        }
        wave_sync_lds();  // column kk scaled
        if (rl > k) {
          const TA lrk = A[r * DIAG_LD + kk];
          for (int c = kk + 1 + h; c <= r; c += 2) A[r * DIAG_LD + c] -= lrk * A[c * DIAG_LD + kk];
        }
        wave_sync_lds();
      }
    }
    __syncthreads();
    const int m = TB - b0 - DB;  // rows below the block
    if (m == 0) break;
    if (tid < m) {  // rows below: solve x L_kb^T = a, one row per thread
      const int r = b0 + DB + tid;
      TA x[DB];
#pragma unroll
      for (int c = 0; c < DB; ++c) x[c] = A[r * DIAG_LD + b0 + c];
#pragma unroll
      for (int c = 0; c < DB; ++c) {
        TA sacc = x[c];
#pragma unroll
        for (int k = 0; k < c; ++k) sacc -= x[k] * A[(b0 + c) * DIAG_LD + b0 + k];
        x[c] = sacc / A[(b0 + c) * DIAG_LD + b0 + c];
      }
#pragma unroll
      for (int c = 0; c < DB; ++c) A[r * DIAG_LD + b0 + c] = x[c];
    }
    __syncthreads();
    // trailing update of the lower triangle below and right of the block, 4 x 4 per thread
    const int m4 = m >> 2;
    for (int t = tid; t < m4 * m4; t += NT) {
      const int bi = t / m4, bj = t - bi * m4;
      if (bj > bi) continue;
      const int r0 = b0 + DB + 4 * bi, c0 = b0 + DB + 4 * bj;
      TA acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = TA(0);
      for (int k = 0; k < DB; ++k) {
        TA ar[4], ac[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ar[u] = A[(r0 + u) * DIAG_LD + b0 + k];
          ac[u] = A[(c0 + u) * DIAG_LD + b0 + k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += ar[u] * ac[v];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (c0 + v <= r0 + u) A[(r0 + u) * DIAG_LD + c0 + v] -= acc[u][v];
    }
    __syncthreads();
  }
  if (bad && tid == 0) a.status[p] = 1;
  // store L_jj and its log-diagonal
  for (int idx = tid; idx < TB * TB; idx += NT) {
    const int r = idx >> 7, c = idx & (TB - 1);
    src[(int64_t)r * rj.ld + c] = c <= r ? (T)A[r * DIAG_LD + c] : T(0);
  }
  {
    double ls = 0.0;
    if (tid < TB && tid < rj.nvalid) ls = log((double)A[tid * DIAG_LD + tid]);
    for (int o = 32; o > 0; o >>= 1) ls += __shfl_xor(ls, o);
    if ((tid & 63) == 0) lsum[tid >> 6] = ls;
  }
  __syncthreads();  // the factor is stored and read before the inverse overwrites it
  if (tid == 0) {
    const double tot = lsum[0] + lsum[1] + lsum[2] + lsum[3];
    a.logdiag[(int64_t)p * a.maxT + a.j] = (a.j >= pd.ld_from) ? tot : 0.0;
  }

  // ---- inverse, diagonal blocks: wave w inverts block w, last column first:
  //   X_jj = 1/L_jj,  X_ij = -X_jj sum_{k=j+1..i} X_ik L_kj
  {
    const int b0 = w * DB, il = lane & 31, h = lane >> 5;
    for (int jj = DB - 1; jj >= 0; --jj) {
      const TA xjj = TA(1) / A[(b0 + jj) * DIAG_LD + b0 + jj];
      TA sacc = TA(0);
      if (il > jj)
        for (int k = jj + 1 + h; k <= il; k += 2) sacc += A[(b0 + il) * DIAG_LD + b0 + k] * A[(b0 + k) * DIAG_LD + b0 + jj];
      sacc += __shfl_xor(sacc, 32);
      wave_sync_lds();  // column jj of L read by every lane
      if (h == 0 && il > jj) A[(b0 + il) * DIAG_LD + b0 + jj] = -xjj * sacc;
      if (lane == 0) A[(b0 + jj) * DIAG_LD + b0 + jj] = xjj;
      wave_sync_lds();
    }
  }
  __syncthreads();
  // ---- inverse, block columns right to left
  for (int jb = DNB - 2; jb >= 0; --jb) {
    const int nb = DNB - 1 - jb;
    for (int e = tid; e < nb * DB * DB; e += NT) {
      const int q = e / (DB * DB), rem = e - q * (DB * DB), i = rem / DB, jc = rem - i * DB;
      const int ib = jb + 1 + q;
      TA sacc = TA(0);
      for (int kb2 = jb + 1; kb2 <= ib; ++kb2) {
        const TA* xr = A + (ib * DB + i) * DIAG_LD + kb2 * DB;
        const TA* lc = A + (kb2 * DB) * DIAG_LD + jb * DB + jc;
#pragma unroll 8
        for (int kk = 0; kk < DB; ++kk) sacc += xr[kk] * lc[kk * DIAG_LD];
      }
      Tt[(q * DB + i) * DT_LD + jc] = sacc;
    }
    __syncthreads();
    for (int e = tid; e < nb * DB * DB; e += NT) {
      const int q = e / (DB * DB), rem = e - q * (DB * DB), i = rem / DB, jc = rem - i * DB;
      const int ib = jb + 1 + q;
      TA sacc = TA(0);
      for (int kk = jc; kk < DB; ++kk) sacc += Tt[(q * DB + i) * DT_LD + kk] * A[(jb * DB + kk) * DIAG_LD + jb * DB + jc];
      A[(ib * DB + i) * DIAG_LD + jb * DB + jc] = -sacc;
    }
    __syncthreads();
  }
  T* inv = a.invdiag + pd.invdiag_off + (int64_t)a.j * TB * TB;
  for (int idx = tid; idx < TB * TB; idx += NT) {
    const int r = idx >> 7, c = idx & (TB - 1);
    inv[idx] = c <= r ? (T)A[r * DIAG_LD + c] : T(0);
  }
}

// ---------------------------------------------------------------------------
// trsm: L_ij = C_ij L_jj^-T (in place) for every item (p, i), i != j
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_trsm(StepArgs<T> a) {
  const int logical = xcd_logical(blockIdx.x, gridDim.x);
  if (logical >= a.nitems) return;
  const WorkItem it = a.items[logical];
  const ProbDesc pd = a.pd[it.p];
  const RowTile<T> ri = a.rt[pd.first + it.tile];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  T* C = ri.panel + (int64_t)(a.j - ri.kbeg) * TB;
  const T* Li = a.invdiag + pd.invdiag_off + (int64_t)a.j * TB * TB;
  typename Mfma<T>::acc acc[4][4];
  zero_acc<T>(acc);
  wave_gemm<T, T>(acc, C, ri.ld, ri.nstore, Li, TB, TB, 0, TB, wr * 64, wc * 64, lane);
  __syncthreads();  // every wave has consumed its reads of C before anyone overwrites it
#pragma unroll
  for (int rs = 0; rs < 4; ++rs)
#pragma unroll
    for (int cs = 0; cs < 4; ++cs)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 64 + rs * 16 + Mfma<T>::row(lane, v);
        const int col = wc * 64 + cs * 16 + (lane & 15);
        if (row < ri.nstore) C[(int64_t)row * ri.ld + col] = acc[rs][cs][v];
      }
}

// ---------------------------------------------------------------------------
// batched float64-accumulating tile GEMM
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_tile_gemm(const GemmTerm<T>* __restrict__ terms,
                                                  const GemmOut* __restrict__ outs, int nout) {
  const int logical = xcd_logical(blockIdx.x, gridDim.x);
  if (logical >= nout) return;
  const GemmOut o = outs[logical];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  typename Mfma<double>::acc acc[4][4];
  zero_acc<double>(acc);
  for (int t = o.t0; t < o.t1; ++t) {
    if (t == o.tneg && t > o.t0) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = -acc[a][b];
    }
    const GemmTerm<T> tm = terms[t];
    wave_gemm<T, double>(acc, tm.a, tm.lda, tm.anr, tm.b, tm.ldb, tm.bnr, tm.k0, tm.k1, wr * 64, wc * 64,
                         lane);
  }
  if (o.tneg == o.t1 && o.t1 > o.t0) {  // only subtracted terms
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = -acc[a][b];
  }
#pragma unroll
  for (int rs = 0; rs < 4; ++rs)
#pragma unroll
    for (int cs = 0; cs < 4; ++cs)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 64 + rs * 16 + Mfma<double>::row(lane, v);
        const int col = wc * 64 + cs * 16 + (lane & 15);
        if (row < o.rows && col < o.cols) {
          double* q = o.out + (int64_t)row * o.ld + col;
          double r = o.alpha * acc[rs][cs][v];
          if (o.c) r += o.beta * o.c[(int64_t)row * o.ldc + col];
          *q = o.accumulate ? *q + r : r;
        }
      }
}

// ---------------------------------------------------------------------------
// band: R_pq = K_pq + [p == q] sn2 - V_p . V_q on one 128 x 128 tile of the
// residual band (float64 arithmetic, one rounding to T on the store)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_band(BandArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int logical = xcd_logical(blockIdx.x, gridDim.x);
  if (logical >= a.nitems) return;
  const BandItem it = a.items[logical];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  // coordinates of the tile's row and column points
  const int d = a.d;
  double* xr = reinterpret_cast<double*>(smem_raw);  // [d][TB]
  double* xc = xr + d * TB;
  for (int idx = tid; idx < TB * d; idx += NT) {
    const int r = idx / d, t = idx - r * d;
    xr[t * TB + r] = r < it.nr ? a.Xr[(it.p0 + r) * d + t] : 0.0;
    xc[t * TB + r] = r < it.nc ? a.Xs[(it.q0 + r) * d + t] : 0.0;
  }
  typename Mfma<double>::acc acc[4][4];
  zero_acc<double>(acc);
  wave_gemm<double, double>(acc, a.Vr + it.p0 * a.vld, a.vld, it.nr, a.Vt + it.q0 * a.vld, a.vld, it.nc, 0, a.vlen,
                            wr * 64, wc * 64, lane);
  __syncthreads();
  // squared distances of the lane's 64 entries, one coordinate at a time (its 16
  // row and 4 column values of a coordinate are read from LDS once)
  double sq[4][4][4];
#pragma unroll
  for (int rs = 0; rs < 4; ++rs)
#pragma unroll
    for (int cs = 0; cs < 4; ++cs)
#pragma unroll
      for (int v = 0; v < 4; ++v) sq[rs][cs][v] = 0.0;
  for (int t = 0; t < d; ++t) {
    double cv[4];
#pragma unroll
    for (int cs = 0; cs < 4; ++cs) cv[cs] = xc[t * TB + wc * 64 + cs * 16 + (lane & 15)];
#pragma unroll
    for (int rs = 0; rs < 4; ++rs)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double rv = xr[t * TB + wr * 64 + rs * 16 + Mfma<double>::row(lane, v)];
#pragma unroll
        for (int cs = 0; cs < 4; ++cs) {
          const double df = rv - cv[cs];
          sq[rs][cs][v] += df * df;
        }
      }
  }
#pragma unroll
  for (int rs = 0; rs < 4; ++rs)
#pragma unroll
    for (int cs = 0; cs < 4; ++cs)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 64 + rs * 16 + Mfma<double>::row(lane, v);
        const int col = wc * 64 + cs * 16 + (lane & 15);
        if (row < it.nr && col < it.nc) {
          double kv = a.sf2 * k_exp(-0.5 * sq[rs][cs][v]);
          if (a.noise && it.p0 + row == it.q0 + col) kv += a.sn2;
          a.band[it.off + (int64_t)row * it.ld + col] = (T)(kv - acc[rs][cs][v]);
        }
      }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int pad8(int n) { return ((n + 7) / 8) * 8; }

template <typename T>
size_t diag_lds_bytes() {
  return sizeof(T) * (size_t)(TB * DIAG_LD + (DNB - 1) * DB * DT_LD);
}

template <typename T>
void launch_update(const StepArgs<T>& a, bool mixed, hipStream_t st) {
  if (a.nitems <= 0) return;
  if constexpr (std::is_same<T, float>::value) {
    if (mixed) {
      const size_t lds = 2 * (size_t)a.d * TB * sizeof(double);
      hipLaunchKernelGGL((k_update<T, true>), dim3(pad8(a.nitems)), dim3(NT), lds, st, a);
      return;
    }
  }
  {
    const size_t lds = 2 * (size_t)a.d * TB * sizeof(T);
    hipLaunchKernelGGL((k_update<T, false>), dim3(pad8(a.nitems)), dim3(NT), lds, st, a);
  }
}

template <typename T>
void launch_diag(const StepArgs<T>& a, const int32_t* plist, int np, hipStream_t st) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_diag<T>, dim3(np), dim3(NT), diag_lds_bytes<double>(), st, a, plist);
}

template <typename T>
void launch_trsm(const StepArgs<T>& a, hipStream_t st) {
  if (a.nitems <= 0) return;
  hipLaunchKernelGGL(k_trsm<T>, dim3(pad8(a.nitems)), dim3(NT), 0, st, a);
}

template <typename T>
void launch_band(const BandArgs<T>& a, hipStream_t st) {
  if (a.nitems <= 0) return;
  hipLaunchKernelGGL(k_band<T>, dim3(pad8(a.nitems)), dim3(NT), 2 * (size_t)a.d * TB * sizeof(double), st, a);
}

template <typename T>
void launch_tile_gemm(const GemmTerm<T>* terms, const GemmOut* outs, int nout, hipStream_t st) {
  if (nout <= 0) return;
  hipLaunchKernelGGL(k_tile_gemm<T>, dim3(pad8(nout)), dim3(NT), 0, st, terms, outs, nout);
}

// Raise the dynamic-LDS limit of the kernels that need more than the default.
hipError_t engine_init() {
  hipError_t e = hipFuncSetAttribute((const void*)k_diag<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)diag_lds_bytes<double>());
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_diag<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)diag_lds_bytes<double>());
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_update<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(2 * 64 * TB * sizeof(double)));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_update<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(2 * 64 * TB * sizeof(double)));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_update<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(2 * 64 * TB * sizeof(float)));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_band<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(2 * 64 * TB * sizeof(double)));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_band<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(2 * 64 * TB * sizeof(double)));
}

template void launch_update<double>(const StepArgs<double>&, bool, hipStream_t);
template void launch_update<float>(const StepArgs<float>&, bool, hipStream_t);
template void launch_diag<double>(const StepArgs<double>&, const int32_t*, int, hipStream_t);
template void launch_diag<float>(const StepArgs<float>&, const int32_t*, int, hipStream_t);
template void launch_trsm<double>(const StepArgs<double>&, hipStream_t);
template void launch_trsm<float>(const StepArgs<float>&, hipStream_t);
template void launch_band<double>(const BandArgs<double>&, hipStream_t);
template void launch_band<float>(const BandArgs<float>&, hipStream_t);
template void launch_tile_gemm<double>(const GemmTerm<double>*, const GemmOut*, int, hipStream_t);
template void launch_tile_gemm<float>(const GemmTerm<float>*, const GemmOut*, int, hipStream_t);

}  // namespace lma
