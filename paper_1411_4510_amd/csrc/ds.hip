// Warm-start network (deep sets) on gfx950: forward, backward and Adam kernels
// and the lma_ds_* C ABI (include/lma_ds.h).
//
// Per-point layers run on the bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16,
// float32 accumulation) with a workgroup of 4 wave64 per 128-point x 128-unit
// tile (wave (wr, wc) owns a 64 x 64 quadrant as 4 x 4 MFMA sub-tiles; lane l
// supplies row l%16 and eight consecutive k starting at 8*(l/16); output
// register v of lane l is row 4*(l/16)+v, column l%16).  Bias, ReLU, the
// per-dataset mean and the head run in float32 on the vector units; every
// reduction has a fixed order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "lma_ds.h"
#include "runtime.h"

namespace lma {
namespace ds {

constexpr int W = 256;          // encoder / head width
constexpr int NF = LMA_DS_NFEAT;
constexpr int KF = 32;          // feature dimension padded for the k=32 MFMA
constexpr int NO = LMA_DS_NOUT;
constexpr int TR = 128;         // points per tile
constexpr int KCH = 4096;       // points per split-K chunk of the weight gradients
// parameter offsets (float32 vector)
constexpr int64_t OW1 = 0, OB1 = OW1 + W * NF, OW2 = OB1 + W, OB2 = OW2 + W * W, OW3 = OB2 + W,
                  OB3 = OW3 + W * W, OW4 = OB3 + W, OB4 = OW4 + NO * W, NP = OB4 + NO;
static_assert(NP == LMA_DS_NPARAM, "parameter count");

typedef unsigned short u16;
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

// round to nearest bfloat16, ties to even
__device__ inline u16 f2bf(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u16)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf2f(u16 h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline bf8 load8(const u16* p) { return __builtin_bit_cast(bf8, *(const uint4*)p); }
__device__ inline bf8 pack8(const u16 (&h)[8]) {
  uint4 q;
  q.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
  q.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
  q.z = (uint32_t)h[4] | ((uint32_t)h[5] << 16);
  q.w = (uint32_t)h[6] | ((uint32_t)h[7] << 16);
  return __builtin_bit_cast(bf8, q);
}
__device__ inline f4v mma(bf8 a, bf8 b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
__device__ inline int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }

__device__ inline void zero(f4v (&acc)[4][4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (f4v){0.f, 0.f, 0.f, 0.f};
}

// acc[ra][rb] += A[arow0 + 16 ra + i][k] * B[brow0 + 16 rb + j][k], k in [k0, k1) (multiples of 32).
// Rows at or past anr / bnr are read from row 0 (callers do not store what they feed).
__device__ inline void wgemm(f4v (&acc)[4][4], const u16* __restrict__ A, int64_t lda, int anr,
                             const u16* __restrict__ B, int64_t ldb, int bnr, int64_t k0, int64_t k1, int arow0,
                             int brow0, int lane) {
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  const u16* pa[4];
  const u16* pb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int ra = arow0 + 16 * t + r16, rb = brow0 + 16 * t + r16;
    pa[t] = A + (int64_t)(ra < anr ? ra : 0) * lda + kq;
    pb[t] = B + (int64_t)(rb < bnr ? rb : 0) * ldb + kq;
  }
  for (int64_t k = k0; k < k1; k += 32) {
    bf8 a[4], b[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      a[t] = load8(pa[t] + k);
      b[t] = load8(pb[t] + k);
    }
#pragma unroll
    for (int ra = 0; ra < 4; ++ra)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) acc[ra][rb] = mma(a[ra], b[rb], acc[ra][rb]);
  }
}

struct Net {
  float* P;      // master parameters [NP]
  float* G;      // gradient [NP]
  float* M1;     // Adam first moment
  float* M2;     // Adam second moment
  u16* W1b;      // [W][KF]  (k >= 17 zero)
  u16* W2b;      // [W][W]
  u16* W2bT;     // [W][W]   transpose of W2b
  u16* W3b;      // [W][W]
  u16* W4b;      // [NO][W]
};

struct Tiles {
  const int32_t* set;    // tile -> dataset
  const int32_t* valid;  // tile -> valid rows (0..128)
  const int64_t* tbeg;   // dataset -> first tile  [nsets+1]
  const float* ninv;     // dataset -> 1 / n_b
};

struct Acts {
  int64_t N;       // rows (multiple of 128)
  u16* H1b;        // [N][W]
  u16* H1bT;       // [W][N]
  u16* FbT;        // [KF][N]
  u16* H2b;        // [N][W]
  float* pool_part;// [ntiles][W]
  float* pool;     // [nsets][W]
  float* z3;       // [nsets][W]
  float* h3;       // [nsets][W]
  float* out;      // [nsets][NO]
  float* dp;       // [nsets][W]   dLoss/dpool, already divided by n_b
  u16* dZ1T;       // [W][N]
  u16* dZ2T;       // [W][N]
  float* wpart;    // split-K partials of dW2 then dW1
  float* hpart;    // per-dataset head partials
  float* lpart;    // per-dataset loss
};

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// Layer 1: H1 = relu(F W1^T + b1) for a 128-point tile and 128 of the units.
__global__ __launch_bounds__(256) void k_l1(Net net, Acts a, Tiles tl, const float* __restrict__ feats) {
  const int t = blockIdx.x >> 1, half = blockIdx.x & 1;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const int nv = tl.valid[t];
  const int64_t row0 = (int64_t)t * TR;
  // A fragments straight from the float32 features (rounded here); invalid rows are zero
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  bf8 af[4];
#pragma unroll
  for (int ra = 0; ra < 4; ++ra) {
    const int r = wr * 64 + ra * 16 + r16;
    u16 h[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = kq + i;
      h[i] = (r < nv && k < NF) ? f2bf(feats[(row0 + r) * NF + k]) : (u16)0;
    }
    af[ra] = pack8(h);
  }
  f4v acc[4][4];
  zero(acc);
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const bf8 bfr = load8(net.W1b + (int64_t)(half * 128 + wc * 64 + rb * 16 + r16) * KF + kq);
#pragma unroll
    for (int ra = 0; ra < 4; ++ra) acc[ra][rb] = mma(af[ra], bfr, acc[ra][rb]);
  }
  const float* b1 = net.P + OB1;
#pragma unroll
  for (int ra = 0; ra < 4; ++ra)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wr * 64 + ra * 16 + out_row(lane, v);
        const int c = half * 128 + wc * 64 + rb * 16 + r16;
        const float z = acc[ra][rb][v] + b1[c];
        const u16 hb = f2bf(z > 0.f ? z : 0.f);
        a.H1b[(row0 + r) * W + c] = hb;
        a.H1bT[(int64_t)c * a.N + row0 + r] = hb;
      }
  if (half == 0) {
    for (int idx = tid; idx < KF * TR; idx += 256) {
      const int k = idx / TR, r = idx - k * TR;
      a.FbT[(int64_t)k * a.N + row0 + r] = (r < nv && k < NF) ? f2bf(feats[(row0 + r) * NF + k]) : (u16)0;
    }
  }
}

// Layer 2: H2 = relu(H1b W2^T + b2); its ReLU pattern (as bfloat16 H2) and the
// tile's column sums over valid rows (fixed order) for the mean.
__global__ __launch_bounds__(256) void k_l2(Net net, Acts a, Tiles tl) {
  __shared__ float red[2][128];
  const int t = blockIdx.x >> 1, half = blockIdx.x & 1;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const int nv = tl.valid[t];
  const int64_t row0 = (int64_t)t * TR;
  f4v acc[4][4];
  zero(acc);
  wgemm(acc, a.H1b + row0 * W, W, TR, net.W2b + (int64_t)half * 128 * W, W, 128, 0, W, wr * 64, wc * 64, lane);
  const float* b2 = net.P + OB2;
  float cs[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ra = 0; ra < 4; ++ra)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wr * 64 + ra * 16 + out_row(lane, v);
        const int c = half * 128 + wc * 64 + rb * 16 + (lane & 15);
        const float z = acc[ra][rb][v] + b2[c];
        const float h = z > 0.f ? z : 0.f;
        a.H2b[(row0 + r) * W + c] = f2bf(h);
        if (r < nv) cs[rb] += h;
      }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    cs[rb] += __shfl_xor(cs[rb], 16);
    cs[rb] += __shfl_xor(cs[rb], 32);
  }
  if (lane < 16)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) red[wr][wc * 64 + rb * 16 + lane] = cs[rb];
  __syncthreads();
  if (tid < 128) a.pool_part[(int64_t)t * W + half * 128 + tid] = red[0][tid] + red[1][tid];
}

// mean over each dataset's tiles (in tile order), then the head in float32
__global__ __launch_bounds__(256) void k_head(Net net, Acts a, Tiles tl) {
  __shared__ float sp[W], sh[W];
  const int b = blockIdx.x, i = threadIdx.x;
  float s = 0.f;
  for (int64_t t = tl.tbeg[b]; t < tl.tbeg[b + 1]; ++t) s += a.pool_part[t * W + i];
  const float p = s * tl.ninv[b];
  a.pool[(int64_t)b * W + i] = p;
  sp[i] = p;
  __syncthreads();
  float z = net.P[OB3 + i];
  for (int k = 0; k < W; ++k) z += bf2f(net.W3b[i * W + k]) * sp[k];
  a.z3[(int64_t)b * W + i] = z;
  const float h = z > 0.f ? z : 0.f;
  a.h3[(int64_t)b * W + i] = h;
  sh[i] = h;
  __syncthreads();
  if (i < NO) {
    float o = net.P[OB4 + i];
    for (int k = 0; k < W; ++k) o += bf2f(net.W4b[i * W + k]) * sh[k];
    a.out[(int64_t)b * NO + i] = o;
  }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// per dataset: output gradient of the masked MSE, head gradients (partials per
// dataset), and dLoss/dpool / n_b
__global__ __launch_bounds__(256) void k_head_bwd(Net net, Acts a, Tiles tl, const float* __restrict__ labels,
                                                  const float* __restrict__ masks, int nsets) {
  __shared__ float sdo[NO], sdz[W];
  const int b = blockIdx.x, i = threadIdx.x;
  float* hp = a.hpart + (int64_t)b * (W * W + W + NO * W + NO);  // W3, b3, W4, b4 partials
  if (i == 0) {
    float cnt = 0.f, l = 0.f;
    for (int j = 0; j < NO; ++j) cnt += masks[b * NO + j];
    for (int j = 0; j < NO; ++j) {
      const float r = (a.out[b * NO + j] - labels[b * NO + j]) * masks[b * NO + j];
      sdo[j] = 2.f * r / cnt / (float)nsets;
      l += r * r;
    }
    a.lpart[b] = l / cnt / (float)nsets;
  }
  __syncthreads();
  const float h3 = a.h3[(int64_t)b * W + i];
  for (int j = 0; j < NO; ++j) hp[W * W + W + j * W + i] = sdo[j] * h3;
  if (i < NO) hp[W * W + W + NO * W + i] = sdo[i];
  float dh = 0.f;
  for (int j = 0; j < NO; ++j) dh += bf2f(net.W4b[j * W + i]) * sdo[j];
  const float dz = a.z3[(int64_t)b * W + i] > 0.f ? dh : 0.f;
  sdz[i] = dz;
  hp[W * W + i] = dz;
  __syncthreads();
  const float* pool = a.pool + (int64_t)b * W;
  for (int r = 0; r < W; ++r) hp[r * W + i] = sdz[r] * pool[i];
  float dpv = 0.f;
  for (int r = 0; r < W; ++r) dpv += bf2f(net.W3b[r * W + i]) * sdz[r];
  a.dp[(int64_t)b * W + i] = dpv * tl.ninv[b];
}

// sum of the per-dataset head partials into the gradient (dataset order)
__global__ void k_head_reduce(Net net, Acts a, int nsets) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nh = W * W + W + NO * W + NO;
  if (e >= nh) return;
  float s = 0.f;
  for (int b = 0; b < nsets; ++b) s += a.hpart[(int64_t)b * nh + e];
  net.G[OW3 + e] = s;  // W3, b3, W4, b4 are contiguous in the parameter vector
}

__global__ void k_loss_reduce(Acts a, int nsets, float* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int b = 0; b < nsets; ++b) s += a.lpart[b];
    *loss = s;
  }
}

// dZ2 = bf16(dp / n * [H2 > 0]) (zero on padding rows); dH1 = dZ2 W2 on the
// matrix cores; dZ1 = bf16(dH1) * [H1 > 0].  Writes dZ1^T, and dZ2^T (half 0).
__global__ __launch_bounds__(256) void k_l2_bwd(Net net, Acts a, Tiles tl) {
  __shared__ float sdp[W];
  const int t = blockIdx.x >> 1, half = blockIdx.x & 1;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const int nv = tl.valid[t];
  const int b = tl.set[t];
  const int64_t row0 = (int64_t)t * TR;
  sdp[tid] = a.dp[(int64_t)b * W + tid];
  __syncthreads();
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  f4v acc[4][4];
  zero(acc);
  for (int k = 0; k < W; k += 32) {
    bf8 af[4], bfr[4];
#pragma unroll
    for (int ra = 0; ra < 4; ++ra) {
      const int r = wr * 64 + ra * 16 + r16;
      const uint4 q = *(const uint4*)(a.H2b + (row0 + r) * W + k + kq);
      const uint32_t qw[4] = {q.x, q.y, q.z, q.w};
      u16 h[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const bool on = ((qw[i >> 1] >> (16 * (i & 1))) & 0xFFFFu) != 0u;
        h[i] = (r < nv && on) ? f2bf(sdp[k + kq + i]) : (u16)0;
      }
      af[ra] = pack8(h);
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
      bfr[rb] = load8(net.W2bT + (int64_t)(half * 128 + wc * 64 + rb * 16 + r16) * W + k + kq);
#pragma unroll
    for (int ra = 0; ra < 4; ++ra)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) acc[ra][rb] = mma(af[ra], bfr[rb], acc[ra][rb]);
  }
#pragma unroll
  for (int ra = 0; ra < 4; ++ra)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wr * 64 + ra * 16 + out_row(lane, v);
        const int c = half * 128 + wc * 64 + rb * 16 + r16;
        const bool on = a.H1b[(row0 + r) * W + c] != 0;
        a.dZ1T[(int64_t)c * a.N + row0 + r] = on ? f2bf(acc[ra][rb][v]) : (u16)0;
      }
  if (half == 0) {
    for (int idx = tid; idx < W * TR; idx += 256) {
      const int o = idx / TR, r = idx - o * TR;
      const bool on = r < nv && a.H2b[(row0 + r) * W + o] != 0;
      a.dZ2T[(int64_t)o * a.N + row0 + r] = on ? f2bf(sdp[o]) : (u16)0;
    }
  }
}

// split-K weight gradients: item (job, row tile, chunk); job 0: dW2 = dZ2^T H1b
// (256 x 256), job 1: dW1 = dZ1^T Fb (256 x 17).  Partials [chunk][256][cols].
__global__ __launch_bounds__(256) void k_wgrad(Net net, Acts a, int nchunk, int64_t rows) {
  const int id = blockIdx.x;
  const int per2 = 2 * 2 * nchunk;  // job 0: 2 row tiles x 2 column tiles x chunks
  int job, ti, tj, c;
  if (id < per2) {
    job = 0;
    c = id / 4;
    ti = (id & 3) >> 1;
    tj = id & 1;
  } else {
    job = 1;
    const int r = id - per2;
    c = r / 2;
    ti = r & 1;
    tj = 0;
  }
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const int64_t k0 = (int64_t)c * KCH, k1 = k0 + KCH < rows ? k0 + KCH : rows;
  const u16* A = (job == 0 ? a.dZ2T : a.dZ1T) + (int64_t)ti * 128 * a.N;
  const u16* B = job == 0 ? a.H1bT + (int64_t)tj * 128 * a.N : a.FbT;
  const int bnr = job == 0 ? 128 : NF;
  const int cols = job == 0 ? W : NF;
  f4v acc[4][4];
  zero(acc);
  wgemm(acc, A, a.N, 128, B, a.N, bnr, k0, k1, wr * 64, wc * 64, lane);
  float* out = a.wpart + (job == 0 ? (int64_t)c * W * W : (int64_t)nchunk * W * W + (int64_t)c * W * NF);
#pragma unroll
  for (int ra = 0; ra < 4; ++ra)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = ti * 128 + wr * 64 + ra * 16 + out_row(lane, v);
        const int cc = tj * 128 + wc * 64 + rb * 16 + (lane & 15);
        if (cc < cols) out[(int64_t)r * cols + cc] = acc[ra][rb][v];
      }
}

// chunk sums of the weight-gradient partials (chunk order) and bias gradients
// as row sums of dZ^T (fixed tree order)
__global__ void k_wgrad_reduce(Net net, Acts a, int nchunk) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)W * W) {
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += a.wpart[(int64_t)c * W * W + e];
    net.G[OW2 + e] = s;
  } else if (e < (int64_t)W * W + W * NF) {
    const int64_t f = e - (int64_t)W * W;
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += a.wpart[(int64_t)nchunk * W * W + (int64_t)c * W * NF + f];
    net.G[OW1 + f] = s;
  }
}

__global__ __launch_bounds__(256) void k_bias_grad(Net net, Acts a, int64_t rows) {
  __shared__ float red[256];
  const int o = blockIdx.x >> 1, job = blockIdx.x & 1, tid = threadIdx.x;
  const u16* row = (job == 0 ? a.dZ2T : a.dZ1T) + (int64_t)o * a.N;
  float s = 0.f;
  for (int64_t n = tid; n < rows; n += 256) s += bf2f(row[n]);
  red[tid] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) red[tid] += red[tid + k];
    __syncthreads();
  }
  if (tid == 0) net.G[(job == 0 ? OB2 : OB1) + o] = red[0];
}

// ---------------------------------------------------------------------------
// Adam and the bfloat16 weight copies
// ---------------------------------------------------------------------------
__global__ void k_adam(Net net, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NP) return;
  const float g = net.G[e];
  const float m = b1 * net.M1[e] + (1.f - b1) * g;
  const float v = b2 * net.M2[e] + (1.f - b2) * g * g;
  net.M1[e] = m;
  net.M2[e] = v;
  net.P[e] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

__global__ void k_shadow(Net net) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)W * KF) {
    const int i = (int)(e / KF), k = (int)(e % KF);
    net.W1b[e] = k < NF ? f2bf(net.P[OW1 + i * NF + k]) : (u16)0;
  }
  if (e < (int64_t)W * W) {
    const int i = (int)(e / W), k = (int)(e % W);
    const u16 h2 = f2bf(net.P[OW2 + e]);
    net.W2b[e] = h2;
    net.W2bT[(int64_t)k * W + i] = h2;
    net.W3b[e] = f2bf(net.P[OW3 + e]);
  }
  if (e < (int64_t)NO * W) net.W4b[e] = f2bf(net.P[OW4 + e]);
}

// ---------------------------------------------------------------------------
// features of one dataset
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ystats(const double* __restrict__ y, int64_t n, double* stats) {
  __shared__ double r1[256], r2[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int64_t i = tid; i < n; i += 256) s += y[i];
  r1[tid] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) r1[tid] += r1[tid + k];
    __syncthreads();
  }
  const double mean = r1[0] / (double)n;
  double q = 0.0;
  for (int64_t i = tid; i < n; i += 256) q += (y[i] - mean) * (y[i] - mean);
  r2[tid] = q;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) r2[tid] += r2[tid + k];
    __syncthreads();
  }
  if (tid == 0) {
    stats[0] = mean;
    stats[1] = 1.0 / sqrt(r2[0] / (double)n);
  }
}

__global__ void k_features(const double* __restrict__ X, const double* __restrict__ y, int64_t n, int d,
                           const double* __restrict__ stats, float* __restrict__ F) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * NF) return;
  const int64_t i = e / NF;
  const int k = (int)(e - i * NF);
  float v;
  if (k < 8) v = k < d ? (float)X[i * d + k] : 0.f;
  else if (k == 8) v = (float)((y[i] - stats[0]) * stats[1]);
  else v = (k - 9) < d ? 1.f : 0.f;
  F[e] = v;
}

}  // namespace ds
}  // namespace lma

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using namespace lma;
using namespace lma::ds;
using lmart::Err;

struct lma_ds {
  int64_t max_rows = 0, max_sets = 0;
  char* mem = nullptr;
  Net net{};
  Acts act{};
  int32_t* d_set = nullptr;
  int32_t* d_valid = nullptr;
  int64_t* d_tbeg = nullptr;
  float* d_ninv = nullptr;
  float* d_loss = nullptr;
  double* d_stats = nullptr;
  int64_t nsets = 0, ntiles = 0, rows = 0;
  int64_t step = 0;
  bool have_fwd = false;
  std::vector<int32_t> h_set, h_valid;
  std::vector<int64_t> h_tbeg;
  std::vector<float> h_ninv;
  ~lma_ds() {
    if (mem) (void)hipFree(mem);
  }
};

namespace {

inline int64_t al(int64_t b) { return (b + 255) / 256 * 256; }
inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

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

lma_status lma_ds_create(int64_t max_rows, int64_t max_sets, lma_ds** out) {
  return guard([&] {
    if (!out) throw Err{LMA_E_ARG, "out is NULL"};
    *out = nullptr;
    if (max_rows < TR || max_sets < 1) throw Err{LMA_E_ARG, "need max_rows >= 128 and max_sets >= 1"};
    std::unique_ptr<lma_ds> s(new lma_ds());
    const int64_t N = (max_rows + TR - 1) / TR * TR;
    const int64_t nt = N / TR, nchunk = (N + KCH - 1) / KCH;
    const int64_t nh = (int64_t)W * W + W + NO * W + NO;
    s->max_rows = N;
    s->max_sets = max_sets;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
      const int64_t o = off;
      off += al(bytes);
      return o;
    };
    const int64_t oP = take(4 * NP), oG = take(4 * NP), oM1 = take(4 * NP), oM2 = take(4 * NP);
    const int64_t oW1 = take(2 * W * KF), oW2 = take(2 * W * W), oW2T = take(2 * W * W), oW3 = take(2 * W * W),
                  oW4 = take(2 * NO * W);
    const int64_t oH1 = take(2 * N * W), oH1T = take(2 * N * W), oFT = take(2 * KF * N), oH2 = take(2 * N * W);
    const int64_t oPP = take(4 * nt * W), oPool = take(4 * max_sets * W), oZ3 = take(4 * max_sets * W),
                  oH3 = take(4 * max_sets * W), oOut = take(4 * max_sets * NO), oDp = take(4 * max_sets * W);
    const int64_t oZ1T = take(2 * N * W), oZ2T = take(2 * N * W);
    const int64_t oWp = take(4 * nchunk * ((int64_t)W * W + W * NF)), oHp = take(4 * max_sets * nh),
                  oLp = take(4 * max_sets);
    const int64_t oSet = take(4 * nt), oVal = take(4 * nt), oTb = take(8 * (max_sets + 1)), oNi = take(4 * max_sets),
                  oLoss = take(8), oStats = take(16);
    void* mem = nullptr;
    if (hipMalloc(&mem, off) != hipSuccess || !mem) {
      (void)hipGetLastError();
      throw Err{LMA_E_NOMEM, "device allocation of the network workspace failed"};
    }
    s->mem = (char*)mem;
    char* b = s->mem;
    HIPCHK(hipMemset(b, 0, off));
    s->net = Net{(float*)(b + oP), (float*)(b + oG), (float*)(b + oM1), (float*)(b + oM2), (u16*)(b + oW1),
                 (u16*)(b + oW2), (u16*)(b + oW2T), (u16*)(b + oW3), (u16*)(b + oW4)};
    Acts& a = s->act;
    a.N = N;
    a.H1b = (u16*)(b + oH1);
    a.H1bT = (u16*)(b + oH1T);
    a.FbT = (u16*)(b + oFT);
    a.H2b = (u16*)(b + oH2);
    a.pool_part = (float*)(b + oPP);
    a.pool = (float*)(b + oPool);
    a.z3 = (float*)(b + oZ3);
    a.h3 = (float*)(b + oH3);
    a.out = (float*)(b + oOut);
    a.dp = (float*)(b + oDp);
    a.dZ1T = (u16*)(b + oZ1T);
    a.dZ2T = (u16*)(b + oZ2T);
    a.wpart = (float*)(b + oWp);
    a.hpart = (float*)(b + oHp);
    a.lpart = (float*)(b + oLp);
    s->d_set = (int32_t*)(b + oSet);
    s->d_valid = (int32_t*)(b + oVal);
    s->d_tbeg = (int64_t*)(b + oTb);
    s->d_ninv = (float*)(b + oNi);
    s->d_loss = (float*)(b + oLoss);
    s->d_stats = (double*)(b + oStats);
    *out = s.release();
  });
}

void lma_ds_free(lma_ds* ds) { delete ds; }

lma_status lma_ds_set_params(lma_ds* ds, const float* params) {
  return guard([&] {
    if (!ds || !params) throw Err{LMA_E_ARG, "NULL argument"};
    HIPCHK(hipMemcpy(ds->net.P, params, 4 * NP, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(ds->net.M1, 0, 4 * NP));
    HIPCHK(hipMemset(ds->net.M2, 0, 4 * NP));
    hipLaunchKernelGGL(k_shadow, dim3(nb((int64_t)W * W)), dim3(256), 0, 0, ds->net);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    ds->step = 0;
  });
}

lma_status lma_ds_get_params(lma_ds* ds, float* params) {
  return guard([&] {
    if (!ds || !params) throw Err{LMA_E_ARG, "NULL argument"};
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(params, ds->net.P, 4 * NP, hipMemcpyDeviceToHost));
  });
}

lma_status lma_ds_features(lma_ds* ds, const double* X, const double* y, int64_t n, int32_t d, float* feats,
                           hipStream_t st) {
  return guard([&] {
    if (!ds || !X || !y || !feats) throw Err{LMA_E_ARG, "NULL argument"};
    if (n < 2 || d < 1 || d > 8) throw Err{LMA_E_ARG, "need n >= 2 and 1 <= d <= 8"};
    hipLaunchKernelGGL(k_ystats, dim3(1), dim3(256), 0, st, y, n, ds->d_stats);
    hipLaunchKernelGGL(k_features, dim3(nb(n * NF)), dim3(256), 0, st, X, y, n, (int)d, ds->d_stats, feats);
    HIPCHK(hipGetLastError());
  });
}

lma_status lma_ds_forward(lma_ds* ds, int64_t nsets, const int64_t* set_ptr, const int64_t* set_n,
                          const float* feats, float* out, hipStream_t st) {
  return guard([&] {
    if (!ds || !set_ptr || !set_n || !feats || !out) throw Err{LMA_E_ARG, "NULL argument"};
    if (nsets < 1 || nsets > ds->max_sets) throw Err{LMA_E_ARG, "nsets out of range"};
    if (set_ptr[0] != 0) throw Err{LMA_E_ARG, "set_ptr[0] must be 0"};
    for (int64_t b = 0; b < nsets; ++b) {
      if (set_ptr[b] % TR) throw Err{LMA_E_ARG, "set_ptr entries must be multiples of 128"};
      if (set_n[b] < 1 || set_ptr[b] + set_n[b] > set_ptr[b + 1])
        throw Err{LMA_E_ARG, "each set needs 1 <= set_n[b] <= set_ptr[b+1] - set_ptr[b]"};
    }
    const int64_t rows = (set_ptr[nsets] + TR - 1) / TR * TR;
    if (rows > ds->max_rows) throw Err{LMA_E_ARG, "more rows than the workspace holds"};
    ds->h_set.clear();
    ds->h_valid.clear();
    ds->h_tbeg.assign(nsets + 1, 0);
    ds->h_ninv.assign(nsets, 0.f);
    for (int64_t b = 0; b < nsets; ++b) {
      ds->h_tbeg[b] = (int64_t)ds->h_set.size();
      const int64_t nt = (set_ptr[b + 1] - set_ptr[b] + TR - 1) / TR;
      for (int64_t t = 0; t < nt; ++t) {
        ds->h_set.push_back((int32_t)b);
        const int64_t v = set_n[b] - t * TR;
        ds->h_valid.push_back((int32_t)(v < 0 ? 0 : (v > TR ? TR : v)));
      }
      ds->h_ninv[b] = 1.0f / (float)set_n[b];
    }
    ds->h_tbeg[nsets] = (int64_t)ds->h_set.size();
    const int64_t ntiles = (int64_t)ds->h_set.size();
    if (ntiles * TR != rows) throw Err{LMA_E_ARG, "set_ptr[nsets] must be a multiple of 128"};
    HIPCHK(hipMemcpyAsync(ds->d_set, ds->h_set.data(), 4 * ntiles, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ds->d_valid, ds->h_valid.data(), 4 * ntiles, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ds->d_tbeg, ds->h_tbeg.data(), 8 * (nsets + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ds->d_ninv, ds->h_ninv.data(), 4 * nsets, hipMemcpyHostToDevice, st));
    ds->nsets = nsets;
    ds->ntiles = ntiles;
    ds->rows = rows;
    Tiles tl{ds->d_set, ds->d_valid, ds->d_tbeg, ds->d_ninv};
    Acts a = ds->act;
    a.N = ds->max_rows;  // row stride of the transposed activations
    hipLaunchKernelGGL(k_l1, dim3(2 * ntiles), dim3(256), 0, st, ds->net, a, tl, feats);
    hipLaunchKernelGGL(k_l2, dim3(2 * ntiles), dim3(256), 0, st, ds->net, a, tl);
    hipLaunchKernelGGL(k_head, dim3(nsets), dim3(256), 0, st, ds->net, a, tl);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, a.out, 4 * NO * nsets, hipMemcpyDeviceToDevice, st));
    ds->have_fwd = true;
  });
}

lma_status lma_ds_backward(lma_ds* ds, const float* labels, const float* masks, float* grad, double* loss,
                           hipStream_t st) {
  return guard([&] {
    if (!ds || !labels || !masks) throw Err{LMA_E_ARG, "NULL argument"};
    if (!ds->have_fwd) throw Err{LMA_E_ARG, "lma_ds_backward needs a preceding lma_ds_forward"};
    Tiles tl{ds->d_set, ds->d_valid, ds->d_tbeg, ds->d_ninv};
    Acts a = ds->act;
    a.N = ds->max_rows;
    const int nsets = (int)ds->nsets;
    const int64_t nh = (int64_t)W * W + W + NO * W + NO;
    hipLaunchKernelGGL(k_head_bwd, dim3(nsets), dim3(256), 0, st, ds->net, a, tl, labels, masks, nsets);
    hipLaunchKernelGGL(k_head_reduce, dim3(nb(nh)), dim3(256), 0, st, ds->net, a, nsets);
    hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(64), 0, st, a, nsets, ds->d_loss);
    hipLaunchKernelGGL(k_l2_bwd, dim3(2 * ds->ntiles), dim3(256), 0, st, ds->net, a, tl);
    // weight gradients: split-K over this batch's rows only (rows beyond it
    // hold values of earlier, larger batches)
    const int nchunk = (int)((ds->rows + KCH - 1) / KCH);
    hipLaunchKernelGGL(k_wgrad, dim3(6 * nchunk), dim3(256), 0, st, ds->net, a, nchunk, ds->rows);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb((int64_t)W * W + W * NF)), dim3(256), 0, st, ds->net, a, nchunk);
    hipLaunchKernelGGL(k_bias_grad, dim3(2 * W), dim3(256), 0, st, ds->net, a, ds->rows);
    HIPCHK(hipGetLastError());
    if (grad) HIPCHK(hipMemcpyAsync(grad, ds->net.G, 4 * NP, hipMemcpyDeviceToDevice, st));
    if (loss) {
      float l = 0.f;
      HIPCHK(hipMemcpyAsync(&l, ds->d_loss, 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      *loss = l;
    }
  });
}

lma_status lma_ds_adam(lma_ds* ds, float lr, float beta1, float beta2, float eps, hipStream_t st) {
  return guard([&] {
    if (!ds) throw Err{LMA_E_ARG, "NULL argument"};
    ds->step += 1;
    const float c1 = 1.f - std::pow(beta1, (float)ds->step), c2 = 1.f - std::pow(beta2, (float)ds->step);
    hipLaunchKernelGGL(k_adam, dim3(nb(NP)), dim3(256), 0, st, ds->net, lr, beta1, beta2, eps, c1, c2);
    hipLaunchKernelGGL(k_shadow, dim3(nb((int64_t)W * W)), dim3(256), 0, st, ds->net);
    HIPCHK(hipGetLastError());
  });
}

}  // extern "C"
