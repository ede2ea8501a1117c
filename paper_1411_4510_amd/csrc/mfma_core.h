// MFMA tile core shared by the engine, the tile GEMM and the gradient
// contraction kernels (gfx950, wave64).
//
// A workgroup of 4 wave64 computes one 128x128 output tile; wave (wr, wc)
// owns the 64x64 quadrant (wr, wc) as 4x4 MFMA 16x16 sub-tiles.  Operand
// fragments are read straight from HBM/L2 in the MFMA 16x16x4 input layout
// (lane l supplies row l%16 and four consecutive k values starting at
// 4*(l/16)); the four MFMA k-steps of a 16-wide k chunk consume those four
// values, so each lane issues one contiguous 4-element load per sub-tile row
// per chunk and the next chunks are prefetched while the current one runs on
// the matrix cores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lma {

typedef double dv4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));

template <typename T>
struct V4;
template <>
struct V4<double> { typedef dv4 type; };
template <>
struct V4<float> { typedef fv4 type; };

template <typename Tc>
struct Mfma;
template <>
struct Mfma<double> {
  typedef dv4 acc;
  __device__ static inline acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // register v of lane l holds row (l/16) + 4v, column l%16 of the 16x16 tile
  __device__ static inline int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef fv4 acc;
  __device__ static inline acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // register v of lane l holds row 4*(l/16) + v, column l%16 of the 16x16 tile
  __device__ static inline int row(int l, int v) { return 4 * (l >> 4) + v; }
};

__device__ inline double k_exp(double x) { return exp(x); }
__device__ inline float k_exp(float x) { return expf(x); }
__device__ inline double k_sqrt(double x) { return sqrt(x); }
__device__ inline float k_sqrt(float x) { return sqrtf(x); }

// Workgroups are dealt round-robin to the 8 XCDs; remap so that consecutive
// work items (tiles of the same problem, which share the B operand) land on
// the same XCD and its L2.  The grid is padded to a multiple of 8.
__device__ inline int xcd_logical(int bid, int nb) {
  const int per = nb >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// acc[ra][rb] += A[arow0 + 16 ra + i, k] * Bm[brow0 + 16 rb + j, k] over k in [k0, k1).
// Rows at or past anr / bnr are read from row 0 instead (always a valid
// address): they only feed output rows / columns that the callers either do
// not store or overwrite with their exact value (padding).  Loads are
// unconditional and rotate through PF+1 register slots, so the chunk in use
// never waits for the chunks in flight.
// PERMA feeds the A rows of each 16-row sub-tile in the order r(4a+b) = a+4b, which
// turns the float32 16x16 output layout into the float64 one (row l/16 + 4v).
// wave_gemm_fold (float32 accumulation, PERMA layout): every FOLD_ITERS steady
// iterations (FOLD_ITERS*(PF+1)*16 k, 144 by default) the float32 accumulators are
// added into the float64 ones and restarted from zero.  A single float32 chain over
// the thousands of k of a late column step loses accuracy linearly in k (about 10x a
// blocked float32 Cholesky at k ~ 3000); chains of 144 are more accurate than one.
constexpr int FOLD_ITERS = 3;
template <typename Tin, typename Tc, bool PERMA, int PF, bool FOLD>
__device__ __forceinline__ void wave_gemm_impl(typename Mfma<Tc>::acc (&acc)[4][4],
                                               const Tin* __restrict__ A, int64_t lda, int anr,
                                               const Tin* __restrict__ Bm, int64_t ldb, int bnr,
                                               int k0, int k1, int arow0, int brow0, int lane,
                                               dv4 (&fold)[4][4]) {
  static_assert(!FOLD || (PERMA && std::is_same<Tc, float>::value), "folding needs the float64 output layout");
  typedef typename V4<Tin>::type vin;
  const int r16 = lane & 15, kq = (lane >> 4) << 2;
  const Tin* pa[4];
  const Tin* pb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int ra = arow0 + t * 16 + (PERMA ? ((r16 >> 2) | ((r16 & 3) << 2)) : r16);
    pa[t] = A + (int64_t)(ra < anr ? ra : 0) * lda + k0 + kq;
    const int rb = brow0 + t * 16 + r16;
    pb[t] = Bm + (int64_t)(rb < bnr ? rb : 0) * ldb + k0 + kq;
  }
  const int nc = (k1 - k0) >> 4;
  if (nc <= 0) return;
  vin sa[PF + 1][4], sb[PF + 1][4];
  // chunk x lives in slot x % (PF+1)
#define LMA_LOAD_CHUNK(X, SLOT)                                \
  {                                                            \
    const int off_ = (X) << 4;                                 \
    const int slot_ = (SLOT);                                  \
    _Pragma("unroll") for (int u_ = 0; u_ < 4; ++u_) {         \
      sa[slot_][u_] = *(const vin*)(pa[u_] + off_);            \
      sb[slot_][u_] = *(const vin*)(pb[u_] + off_);            \
    }                                                          \
  }
#define LMA_MMA_SLOT(SLOT)                                                                 \
  {                                                                                        \
    const int slot_ = (SLOT);                                                              \
    _Pragma("unroll") for (int e = 0; e < 4; ++e) {                                        \
      _Pragma("unroll") for (int ra = 0; ra < 4; ++ra) {                                   \
        _Pragma("unroll") for (int rb = 0; rb < 4; ++rb) {                                 \
          acc[ra][rb] = Mfma<Tc>::op((Tc)sa[slot_][ra][e], (Tc)sb[slot_][rb][e], acc[ra][rb]); \
        }                                                                                  \
      }                                                                                    \
    }                                                                                      \
  }
#define LMA_FOLD()                                                                    \
  if constexpr (FOLD) {                                                              \
    _Pragma("unroll") for (int a_ = 0; a_ < 4; ++a_) {                               \
      _Pragma("unroll") for (int b_ = 0; b_ < 4; ++b_) {                             \
        _Pragma("unroll") for (int v_ = 0; v_ < 4; ++v_) {                           \
          fold[a_][b_][v_] += (double)acc[a_][b_][v_];                               \
          acc[a_][b_][v_] = Tc(0);                                                   \
        }                                                                            \
      }                                                                              \
    }                                                                                \
  }
#pragma unroll
  for (int p = 0; p < PF; ++p)
    if (p < nc) LMA_LOAD_CHUNK(p, p)
  int c = 0;
  int since_fold = 0;
  // steady state: every prefetch is in range, no branches in the body
  for (; c + 2 * PF < nc; c += PF + 1) {
#pragma unroll
    for (int q = 0; q <= PF; ++q) {
      LMA_LOAD_CHUNK(c + q + PF, (q + PF) % (PF + 1))
      LMA_MMA_SLOT(q)
    }
    if constexpr (FOLD) {
      if (++since_fold == FOLD_ITERS) {
        since_fold = 0;
        LMA_FOLD()
      }
    }
  }
  // tail: at most 2*PF+1 chunks, slots known at compile time
#pragma unroll
  for (int t = 0; t <= 2 * PF; ++t) {
    if (c + t < nc) {
      if (c + t + PF < nc) LMA_LOAD_CHUNK(c + t + PF, (t + PF) % (PF + 1))
      LMA_MMA_SLOT(t % (PF + 1))
    }
  }
  LMA_FOLD()
#undef LMA_LOAD_CHUNK
#undef LMA_MMA_SLOT
#undef LMA_FOLD
}

template <typename Tin, typename Tc, bool PERMA = false, int PF = 2>
__device__ __forceinline__ void wave_gemm(typename Mfma<Tc>::acc (&acc)[4][4],
                                          const Tin* __restrict__ A, int64_t lda, int anr,
                                          const Tin* __restrict__ Bm, int64_t ldb, int bnr,
                                          int k0, int k1, int arow0, int brow0, int lane) {
  dv4 unused[4][4];
  wave_gemm_impl<Tin, Tc, PERMA, PF, false>(acc, A, lda, anr, Bm, ldb, bnr, k0, k1, arow0, brow0, lane, unused);
}

// float32 products (PERMA layout) with the sums folded into the float64 accumulators fold
template <int PF = 2>
__device__ __forceinline__ void wave_gemm_fold(fv4 (&acc)[4][4], const float* __restrict__ A, int64_t lda, int anr,
                                               const float* __restrict__ Bm, int64_t ldb, int bnr, int k0, int k1,
                                               int arow0, int brow0, int lane, dv4 (&fold)[4][4]) {
  wave_gemm_impl<float, float, true, PF, true>(acc, A, lda, anr, Bm, ldb, bnr, k0, k1, arow0, brow0, lane, fold);
}

// Accumulators start as the result of an MFMA of zero operands (exactly +0):
// started from constant zeros, the compiler keeps the loop-carried accumulators
// of a k loop in vector registers and copies all of them into the accumulation
// registers and back on every iteration; an MFMA result stays in place.
template <typename Tc>
__device__ inline void zero_acc(typename Mfma<Tc>::acc (&acc)[4][4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<Tc>::op(Tc(0), Tc(0), (typename Mfma<Tc>::acc){Tc(0), Tc(0), Tc(0), Tc(0)});
}


}  // namespace lma
