// Block partition of the inputs on gfx950 (include/lma_part.h): k-means++
// seeding, capacity-bounded assignment, and the composed partition call that
// returns block-contiguous permutations of the training and test points.
//
// Every decision is taken on exact quantities, so results equal a plain
// sequential evaluation bit for bit whatever the scheduling:
//   - squared distances are summed over the coordinates in increasing order
//     with separately rounded products and sums (no fused multiply-add), as in
//     the k-means kernels;
//   - seeding draws with integer weights (squared distances scaled by a power
//     of two and truncated), so block sums and prefix sums are exact in uint64;
//   - the bounded assignment keeps, per centre, the r smallest proposers under
//     the total order (squared distance, point index), found by a radix
//     select on the (float64 bit pattern, index) pair: non-negative doubles
//     order like their bit patterns.
//
// Seeding: per round one kernel updates each point's distance to its nearest
// chosen centre and the block maxima, one workgroup derives the power-of-two
// scale from the maximum, one kernel forms the block sums of the weights, and
// one workgroup finds the drawn point (a scan of the block sums, then of the
// weights of one block).  No host synchronisation between rounds.
//
// Bounded assignment, upper bound: rounds of (propose to the nearest open
// centre, counting sort of the proposers by centre, one workgroup per centre
// selecting its r nearest proposers, accept).  The host reads the number of
// points left after each round.  Lower bound, for each centre c below lo in
// increasing index: the points of centres holding more than lo are the
// candidates; the walk that moves the nearest candidate to c one at a time
// (a donor stops giving at lo) takes exactly the `need` smallest of the union
// of each donor's (count - lo) nearest candidates, so it is two selects: one
// per donor, one over that union.
//
// Permutation: a stable least-significant-digit radix sort of the block keys
// (8-bit digits, one or two passes), chunks of 1024 points with per-chunk digit
// histograms and in-chunk ranks among equal digits, so points of one block keep
// their index order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <string>
#include <vector>

#include "lma_part.h"
#include "misc.h"
#include "runtime.h"

namespace lma {
namespace partk {

constexpr int NT = 256;          // threads per workgroup
constexpr int CG = 8;            // centres per pass of the proposal kernel
constexpr int SORT_CHUNK = 1024; // points per chunk of the radix sort
constexpr uint64_t KEY_ALL = ~(uint64_t)0;

__device__ __forceinline__ double sqdist(const double* __restrict__ p, const double* __restrict__ c, int d) {
#pragma clang fp contract(off)
  double acc = 0.0;
  for (int t = 0; t < d; ++t) {
    const double df = p[t] - c[t];
    const double sq = df * df;
    acc = acc + sq;
  }
  return acc;
}

__device__ __forceinline__ uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }

// key order: (distance bits, index) lexicographic
__device__ __forceinline__ bool key_le(uint64_t k, int64_t i, uint64_t tk, int64_t ti) {
  return k < tk || (k == tk && i <= ti);
}

// ---------------------------------------------------------------------------
// block-wide helpers (NT threads)
// ---------------------------------------------------------------------------
__device__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ uint64_t block_sum_u64(uint64_t v, uint64_t* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const uint64_t r = sh[0];
  __syncthreads();
  return r;
}

// inclusive scan of one uint64 per thread (Hillis-Steele in LDS)
__device__ uint64_t block_incl_scan_u64(uint64_t v, uint64_t* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 1; s < NT; s <<= 1) {
    const uint64_t add = (int)threadIdx.x >= s ? sh[threadIdx.x - s] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  const uint64_t r = sh[threadIdx.x];
  __syncthreads();
  return r;
}

// floor(r * T / 2^32) for T < 2^63, exactly
__device__ __forceinline__ uint64_t scaled_target(uint32_t r, uint64_t T) {
  const uint64_t lo = (uint64_t)r * (T & 0xffffffffull);
  const uint64_t hi = (uint64_t)r * (T >> 32);
  return hi + (lo >> 32);
}

__device__ __forceinline__ uint64_t weight_of(double dmin, int shift, int zero) {
  if (zero) return 0;
  return (uint64_t)floor(ldexp(dmin, shift));
}

// ---------------------------------------------------------------------------
// seeding
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_seed_dmin(const double* __restrict__ P, int64_t n, int d,
                                                  const int64_t* __restrict__ sidx, int j, double* __restrict__ dmin,
                                                  double* __restrict__ bmax) {
  __shared__ double sh[NT];
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const double q = sqdist(P + i * d, P + sidx[j] * d, d);
    const double old = dmin[i];
    v = (j == 0 || q < old) ? q : old;
    dmin[i] = v;
  }
  const double m = block_max(v, sh);
  if (threadIdx.x == 0) bmax[blockIdx.x] = m;
}

// scal[0] = shift W - e, scal[1] = 1 when every weight is 0, scal[2] |= 1 on a
// non-finite maximum
__global__ __launch_bounds__(NT) void k_seed_scale(const double* __restrict__ bmax, int64_t nb, int wbits,
                                                   int32_t* __restrict__ scal) {
  __shared__ double sh[NT];
  double m = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += NT) m = fmax(m, bmax[b]);
  m = block_max(m, sh);
  if (threadIdx.x == 0) {
    if (!isfinite(m)) {
      scal[2] = 1;
      scal[1] = 1;
      scal[0] = 0;
    } else if (!(m > 0.0)) {
      scal[1] = 1;
      scal[0] = 0;
    } else {
      int e = 0;
      (void)frexp(m, &e);
      scal[0] = wbits - e;
      scal[1] = 0;
    }
  }
}

__global__ __launch_bounds__(NT) void k_seed_wsum(const double* __restrict__ dmin, int64_t n,
                                                  const int32_t* __restrict__ scal, uint64_t* __restrict__ bsum) {
  __shared__ uint64_t sh[NT];
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  const uint64_t w = i < n ? weight_of(dmin[i], scal[0], scal[1]) : 0;
  const uint64_t s = block_sum_u64(w, sh);
  if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

// one workgroup: the drawn point of round j
__global__ __launch_bounds__(NT) void k_seed_pick(const double* __restrict__ dmin, int64_t n,
                                                  const int32_t* __restrict__ scal,
                                                  const uint64_t* __restrict__ bsum, int64_t nb,
                                                  const uint32_t* __restrict__ rnd, int j,
                                                  int64_t* __restrict__ sidx) {
  __shared__ uint64_t sh[NT];
  __shared__ int64_t found_b;
  __shared__ uint64_t found_rest;
  // per-thread contiguous ranges of blocks
  const int64_t per = (nb + NT - 1) / NT;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = b0 + per < nb ? b0 + per : nb;
  uint64_t mine = 0;
  for (int64_t b = b0; b < b1; ++b) mine += bsum[b];
  const uint64_t incl = block_incl_scan_u64(mine, sh);
  const uint64_t T = sh[NT - 1];
  __syncthreads();
  const uint32_t r = rnd[j];
  if (T == 0) {
    if (threadIdx.x == 0) sidx[j] = (int64_t)(((uint64_t)r * (uint64_t)n) >> 32);
    return;
  }
  const uint64_t target = scaled_target(r, T);
  if (threadIdx.x == 0) found_b = -1;
  __syncthreads();
  const uint64_t excl = incl - mine;
  if (excl <= target && target < incl) {
    // this thread's range holds the block whose running sum passes the target
    uint64_t run = excl;
    for (int64_t b = b0; b < b1; ++b) {
      if (run + bsum[b] > target) {
        found_b = b;
        found_rest = target - run;
        break;
      }
      run += bsum[b];
    }
  }
  __syncthreads();
  const int64_t b = found_b;
  const uint64_t rest = found_rest;
  const int64_t i = b * NT + threadIdx.x;
  const uint64_t w = (b >= 0 && i < n) ? weight_of(dmin[i], scal[0], scal[1]) : 0;
  const uint64_t wi = block_incl_scan_u64(w, sh);
  if (b >= 0 && wi > rest && wi - w <= rest) sidx[j] = i;
}

__global__ void k_gather_rows(const double* __restrict__ P, int d, const int64_t* __restrict__ idx, int k,
                              double* __restrict__ C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * d) return;
  const int64_t r = e / d, t = e - r * d;
  C[e] = P[idx[r] * d + t];
}

// ---------------------------------------------------------------------------
// bounded assignment
// ---------------------------------------------------------------------------
// Every point without a centre proposes to its nearest centre holding fewer
// than hi points (ties to the lower index).
__global__ __launch_bounds__(NT) void k_propose(const double* __restrict__ P, int64_t n, int d,
                                                const double* __restrict__ C, int k, int64_t hi,
                                                const int64_t* __restrict__ cnt, const int32_t* __restrict__ label,
                                                int32_t* __restrict__ tgt, double* __restrict__ key,
                                                unsigned long long* __restrict__ pcnt) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n || label[i] >= 0) return;
  const double* p = P + i * d;
  double best = INFINITY;
  int arg = -1;
  for (int c0 = 0; c0 < k; c0 += CG) {
    const int nc = k - c0 < CG ? k - c0 : CG;
    double acc[CG];
#pragma unroll
    for (int jj = 0; jj < CG; ++jj) acc[jj] = 0.0;
    const double* cb = C + (int64_t)c0 * d;
    for (int t = 0; t < d; ++t) {
      const double x = p[t];
#pragma unroll
      for (int jj = 0; jj < CG; ++jj) {
        if (jj < nc) {
          const double df = x - cb[jj * d + t];
          const double sq = df * df;
          acc[jj] = acc[jj] + sq;
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < CG; ++jj)
      if (jj < nc && cnt[c0 + jj] < hi && (arg < 0 || acc[jj] < best)) {
        best = acc[jj];
        arg = c0 + jj;
      }
  }
  tgt[i] = arg;
  key[i] = best;
  if (arg >= 0) atomicAdd(&pcnt[arg], 1ull);  // an open centre exists while points are left
}

// One workgroup: segment offsets from the per-segment counts (which it then
// clears), cursors cleared, and each segment's rank: mode 0 = hi - cnt (room
// of a centre), mode 1 = cnt - lo (what a donor can give).
__global__ __launch_bounds__(1024) void k_seg_offsets(unsigned long long* __restrict__ pcnt, int k,
                                                      int64_t* __restrict__ seg_ptr,
                                                      unsigned long long* __restrict__ cursor,
                                                      const int64_t* __restrict__ cnt, int64_t bound, int mode,
                                                      int64_t* __restrict__ rank) {
  __shared__ int64_t sh[1024];
  const int per = (k + 1023) / 1024;
  const int c0 = threadIdx.x * per, c1 = c0 + per < k ? c0 + per : k;
  int64_t mine = 0;
  for (int c = c0; c < c1; ++c) mine += (int64_t)pcnt[c];
  sh[threadIdx.x] = mine;
  __syncthreads();
  for (int s = 1; s < 1024; s <<= 1) {
    const int64_t add = (int)threadIdx.x >= s ? sh[threadIdx.x - s] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t run = sh[threadIdx.x] - mine;
  for (int c = c0; c < c1; ++c) {
    seg_ptr[c] = run;
    run += (int64_t)pcnt[c];
    pcnt[c] = 0;
    cursor[c] = 0;
    rank[c] = mode == 0 ? bound - cnt[c] : cnt[c] - bound;
  }
  if (threadIdx.x == 1023) seg_ptr[k] = sh[1023];
}

// Proposers (tgt >= 0 among points flagged by label < 0, or every point with
// tgt >= 0 when all_tgt) into their segment.
__global__ __launch_bounds__(NT) void k_scatter(int64_t n, const int32_t* __restrict__ label, int all_tgt,
                                                const int32_t* __restrict__ tgt, const double* __restrict__ key,
                                                const int64_t* __restrict__ seg_ptr,
                                                unsigned long long* __restrict__ cursor,
                                                uint64_t* __restrict__ skey, int64_t* __restrict__ sidx) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  if (!all_tgt && label[i] >= 0) return;
  const int c = tgt[i];
  if (c < 0) return;
  const int64_t pos = seg_ptr[c] + (int64_t)atomicAdd(&cursor[c], 1ull);
  skey[pos] = dbits(key[i]);
  sidx[pos] = i;
}

// One workgroup per segment: the rank-th smallest (key, index) of the
// segment, by a most-significant-digit radix select over the 64 key bits and
// then the 64 index bits.  rank <= 0: nothing is taken (threshold below every
// key); rank >= size: everything.
__global__ __launch_bounds__(NT) void k_seg_select(const int64_t* __restrict__ seg_ptr,
                                                   const uint64_t* __restrict__ skey,
                                                   const int64_t* __restrict__ sidx,
                                                   const int64_t* __restrict__ rank, int nseg,
                                                   uint64_t* __restrict__ thr_key, int64_t* __restrict__ thr_idx) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix;
  __shared__ int64_t s_rank;
  const int sg = blockIdx.x;
  if (sg >= nseg) return;
  const int64_t a = seg_ptr[sg], m = seg_ptr[sg + 1] - a;
  const int64_t r0 = rank[sg];
  if (r0 <= 0) {
    if (threadIdx.x == 0) {
      thr_key[sg] = 0;
      thr_idx[sg] = -1;
    }
    return;
  }
  if (r0 >= m) {
    if (threadIdx.x == 0) {
      thr_key[sg] = KEY_ALL;
      thr_idx[sg] = INT64_MAX;
    }
    return;
  }
  if (threadIdx.x == 0) {
    s_prefix = 0;
    s_rank = r0;
  }
  __syncthreads();
  uint64_t kstar = 0;
  // 16 passes: 8 over the key's bytes, 8 over the index's, high byte first
  for (int pass = 0; pass < 16; ++pass) {
    const bool on_key = pass < 8;
    const int shift = 56 - 8 * (pass & 7);
    const uint64_t himask = shift == 56 ? 0 : (~(uint64_t)0 << (shift + 8));
    for (int b = threadIdx.x; b < 256; b += NT) hist[b] = 0;
    __syncthreads();
    const uint64_t prefix = s_prefix;
    for (int64_t e = threadIdx.x; e < m; e += NT) {
      const uint64_t kv = skey[a + e];
      uint64_t v;
      if (on_key) {
        if ((kv & himask) != prefix) continue;
        v = kv;
      } else {
        if (kv != kstar) continue;
        v = (uint64_t)sidx[a + e];
        if ((v & himask) != prefix) continue;
      }
      atomicAdd(&hist[(v >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t need = s_rank;
      int bin = 0;
      for (; bin < 255; ++bin) {
        if ((int64_t)hist[bin] >= need) break;
        need -= hist[bin];
      }
      s_rank = need;
      s_prefix = prefix | ((uint64_t)bin << shift);
    }
    __syncthreads();
    if (pass == 7) {
      kstar = s_prefix;
      __syncthreads();
      if (threadIdx.x == 0) s_prefix = 0;
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    thr_key[sg] = kstar;
    thr_idx[sg] = (int64_t)s_prefix;
  }
}

// Proposers within their centre's threshold join it.
__global__ __launch_bounds__(NT) void k_accept(int64_t n, int32_t* __restrict__ label, const int32_t* __restrict__ tgt,
                                               const double* __restrict__ key, const uint64_t* __restrict__ thr_key,
                                               const int64_t* __restrict__ thr_idx) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n || label[i] >= 0) return;
  const int c = tgt[i];
  if (key_le(dbits(key[i]), i, thr_key[c], thr_idx[c])) label[i] = c;
}

// One workgroup: counts after a round (each centre took min(proposers, room)),
// and the number of points still without a centre.
__global__ __launch_bounds__(1024) void k_round_end(int k, const int64_t* __restrict__ seg_ptr, int64_t hi,
                                                    int64_t* __restrict__ cnt, int64_t* __restrict__ left) {
  __shared__ int64_t sh[1024];
  int64_t took = 0;
  for (int c = threadIdx.x; c < k; c += 1024) {
    const int64_t prop = seg_ptr[c + 1] - seg_ptr[c];
    const int64_t room = hi - cnt[c];
    const int64_t t = prop < room ? prop : room;
    cnt[c] += t;
    took += t;
  }
  sh[threadIdx.x] = took;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) left[0] -= sh[0];
}

// Lower bound, centre c: candidates are the points of centres holding more
// than lo; their key is the squared distance to c, tgt their donor.
__global__ __launch_bounds__(NT) void k_lb_keys(const double* __restrict__ P, int64_t n, int d,
                                                const double* __restrict__ C, int c, const int32_t* __restrict__ label,
                                                const int64_t* __restrict__ cnt, int64_t lo,
                                                int32_t* __restrict__ tgt, double* __restrict__ key,
                                                unsigned long long* __restrict__ pcnt) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int o = label[i];
  if (o == c || cnt[o] <= lo) {
    tgt[i] = -1;
    return;
  }
  tgt[i] = o;
  key[i] = sqdist(P + i * d, C + (int64_t)c * d, d);
  atomicAdd(&pcnt[o], 1ull);
}

// The union A of each donor's (count - lo) nearest candidates, compacted.
__global__ __launch_bounds__(NT) void k_lb_gather(int64_t n, const int32_t* __restrict__ tgt,
                                                  const double* __restrict__ key, const uint64_t* __restrict__ thr_key,
                                                  const int64_t* __restrict__ thr_idx, uint64_t* __restrict__ akey,
                                                  int64_t* __restrict__ aidx, unsigned long long* __restrict__ acount) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int o = tgt[i];
  if (o < 0) return;
  const uint64_t kb = dbits(key[i]);
  if (!key_le(kb, i, thr_key[o], thr_idx[o])) return;
  const int64_t pos = (int64_t)atomicAdd(acount, 1ull);
  akey[pos] = kb;
  aidx[pos] = i;
}

// One thread: segment [0, |A|) and its rank lo - cnt[c].
__global__ void k_lb_seg(const unsigned long long* __restrict__ acount, const int64_t* __restrict__ cnt, int c,
                         int64_t lo, int64_t* __restrict__ aptr, int64_t* __restrict__ arank) {
  aptr[0] = 0;
  aptr[1] = (int64_t)acount[0];
  arank[0] = lo - cnt[c];
}

__global__ __launch_bounds__(NT) void k_lb_move(int64_t n, int c, int32_t* __restrict__ label,
                                                const int32_t* __restrict__ tgt, const double* __restrict__ key,
                                                const uint64_t* __restrict__ thr_key,
                                                const int64_t* __restrict__ thr_idx,
                                                const uint64_t* __restrict__ athr_key,
                                                const int64_t* __restrict__ athr_idx,
                                                unsigned long long* __restrict__ cnt_u) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int o = tgt[i];
  if (o < 0) return;
  const uint64_t kb = dbits(key[i]);
  if (!key_le(kb, i, thr_key[o], thr_idx[o]) || !key_le(kb, i, athr_key[0], athr_idx[0])) return;
  label[i] = c;
  atomicAdd(&cnt_u[o], ~0ull);  // -1
}

__global__ void k_lb_fix(int64_t* __restrict__ cnt, int c, int64_t lo, unsigned long long* __restrict__ acount) {
  cnt[c] = lo;
  acount[0] = 0;
}

// ---------------------------------------------------------------------------
// stable radix sort of block keys (values: point indices)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_digit_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                   int64_t nch, uint32_t* __restrict__ H) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t ch = blockIdx.x;
  for (int s = 0; s < SORT_CHUNK; s += NT) {
    const int64_t i = ch * SORT_CHUNK + s + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  H[(int64_t)threadIdx.x * nch + ch] = h[threadIdx.x];
}

// one workgroup: exclusive scan of H in (digit, chunk) order, in place
__global__ __launch_bounds__(1024) void k_hist_scan(uint32_t* __restrict__ H, int64_t total) {
  __shared__ uint64_t sh[1024];
  const int64_t per = (total + 1023) / 1024;
  const int64_t a = (int64_t)threadIdx.x * per, b = a + per < total ? a + per : total;
  uint64_t mine = 0;
  for (int64_t e = a; e < b; ++e) mine += H[e];
  sh[threadIdx.x] = mine;
  __syncthreads();
  for (int s = 1; s < 1024; s <<= 1) {
    const uint64_t add = (int)threadIdx.x >= s ? sh[threadIdx.x - s] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  uint64_t run = sh[threadIdx.x] - mine;
  for (int64_t e = a; e < b; ++e) {
    const uint32_t v = H[e];
    H[e] = (uint32_t)run;
    run += v;
  }
}

__global__ __launch_bounds__(NT) void k_digit_scatter(const uint32_t* __restrict__ kin, const int64_t* __restrict__ vin,
                                                      int64_t n, int shift, int64_t nch,
                                                      const uint32_t* __restrict__ H, uint32_t* __restrict__ kout,
                                                      int64_t* __restrict__ vout) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t dig[NT];
  const int64_t ch = blockIdx.x;
  run[threadIdx.x] = 0;
  __syncthreads();
  for (int s = 0; s < SORT_CHUNK; s += NT) {
    const int64_t i = ch * SORT_CHUNK + s + threadIdx.x;
    const bool ok = i < n;
    const uint32_t kv = ok ? kin[i] : 0;
    const uint32_t dg = ok ? ((kv >> shift) & 255u) : 256u;
    dig[threadIdx.x] = dg;
    __syncthreads();
    uint32_t before = 0;
    for (int t = 0; t < (int)threadIdx.x; ++t) before += dig[t] == dg ? 1u : 0u;
    if (ok) {
      const int64_t pos = (int64_t)H[(int64_t)dg * nch + ch] + run[dg] + before;
      kout[pos] = kv;
      vout[pos] = vin ? vin[i] : i;
    }
    __syncthreads();
    if (ok) atomicAdd(&run[dg], 1u);
    __syncthreads();
  }
}

__global__ void k_block_keys(const int32_t* __restrict__ label, const int32_t* __restrict__ rank, int64_t n,
                             uint32_t* __restrict__ keys, unsigned long long* __restrict__ bcount) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t b = rank[label[i]];
  keys[i] = (uint32_t)b;
  atomicAdd(&bcount[b], 1ull);
}

// non-finite flag over an array
__global__ void k_nonfinite(const double* __restrict__ a, int64_t n, int32_t* __restrict__ flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(a[i])) flag[0] = 1;
}

}  // namespace partk
}  // namespace lma

namespace {

using lmart::Err;
using namespace lma::partk;

constexpr int MAX_K = 65536;

int64_t nblocks(int64_t n) { return (n + NT - 1) / NT; }

void chk() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Err{LMA_E_HIP, std::string("partition kernel launch: ") + hipGetErrorString(e)};
}

void sync(hipStream_t st) {
  const hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) throw Err{LMA_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e)};
}

int weight_bits(int64_t n) {
  int bl = 0;
  while (bl < 63 && (n >> bl) != 0) ++bl;
  return 63 - bl;
}

// Device workspace from the library's cache, carved into pieces; returned
// after a stream synchronisation.
struct Work {
  char* base = nullptr;
  size_t bytes = 0, used = 0;
  hipStream_t st = nullptr;
  size_t take(size_t b) {
    const size_t off = used;
    used += (b + 255) & ~(size_t)255;
    return off;
  }
  template <class T>
  T* at(size_t off) {
    return reinterpret_cast<T*>(base + off);
  }
  void get(hipStream_t s) {
    st = s;
    bytes = std::max<size_t>(used, 256);
    base = static_cast<char*>(lmart::devcache::get(bytes));
    if (!base) throw Err{LMA_E_NOMEM, "device allocation of the partition workspace failed"};
  }
  ~Work() {
    if (base) {
      (void)hipStreamSynchronize(st);
      lmart::devcache::put(base, bytes);
    }
  }
};

void check_pts(const double* P, int64_t n, int32_t d, const char* what) {
  if (n < 0) throw Err{LMA_E_ARG, std::string(what) + ": n < 0"};
  if (d < 1 || d > lma::MAX_D) throw Err{LMA_E_ARG, "need 1 <= d <= 64"};
  if (n > 0 && !P) throw Err{LMA_E_ARG, std::string(what) + " is NULL"};
  if (n > ((int64_t)1 << 38)) throw Err{LMA_E_ARG, std::string(what) + ": too many points"};
}

void check_finite(const double* a, int64_t n, int32_t* flag, hipStream_t st, const char* what) {
  if (n <= 0) return;
  int32_t h = 0;
  HIPCHK(hipMemsetAsync(flag, 0, 4, st));
  hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)std::min<int64_t>(nblocks(n), 65536)), dim3(NT), 0, st, a, n, flag);
  chk();
  HIPCHK(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, st));
  sync(st);
  if (h) throw Err{LMA_E_ARG, std::string(what) + " holds a non-finite value"};
}

// k-means++ seeding: indices into sidx (device [k]), centres into C (device
// [k][d]); ws pieces: dmin [n], bmax/bsum [nb], scal [3], rnd [k].
void seed(const double* P, int64_t n, int32_t d, int32_t k, const uint32_t* rand_h, double* C, int64_t* sidx,
          double* dmin, double* bmax, uint64_t* bsum, int32_t* scal, uint32_t* rnd, hipStream_t st) {
  const int64_t nb = nblocks(n);
  const int64_t first = (int64_t)(((uint64_t)rand_h[0] * (uint64_t)n) >> 32);
  HIPCHK(hipMemcpyAsync(rnd, rand_h, 4 * (size_t)k, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(sidx, 0, 8 * (size_t)k, st));  // every index valid before it is drawn
  HIPCHK(hipMemcpyAsync(sidx, &first, 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(scal, 0, 12, st));
  const int wb = weight_bits(n);
  for (int j = 0; j < k; ++j) {
    if (j > 0) {
      hipLaunchKernelGGL(k_seed_scale, dim3(1), dim3(NT), 0, st, bmax, nb, wb, scal);
      chk();
      hipLaunchKernelGGL(k_seed_wsum, dim3((unsigned)nb), dim3(NT), 0, st, dmin, n, scal, bsum);
      chk();
      hipLaunchKernelGGL(k_seed_pick, dim3(1), dim3(NT), 0, st, dmin, n, scal, bsum, nb, rnd, j, sidx);
      chk();
    }
    if (j < k - 1) {
      hipLaunchKernelGGL(k_seed_dmin, dim3((unsigned)nb), dim3(NT), 0, st, P, n, (int)d, sidx, j, dmin, bmax);
      chk();
    }
  }
  const int64_t kd = (int64_t)k * d;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((kd + NT - 1) / NT)), dim3(NT), 0, st, P, (int)d, sidx, (int)k, C);
  chk();
  int32_t h[3];
  HIPCHK(hipMemcpyAsync(h, scal, 12, hipMemcpyDeviceToHost, st));
  sync(st);
  if (h[2]) throw Err{LMA_E_ARG, "squared distances overflow float64 in the seeding"};
}

struct BoundedWs {
  int32_t* tgt;
  double* key;
  uint64_t* skey;
  int64_t* sidx;
  uint64_t* akey;
  int64_t* aidx;
  int64_t* cnt;
  unsigned long long* pcnt;
  unsigned long long* cursor;
  int64_t* seg_ptr;
  int64_t* rank;
  uint64_t* thr_key;
  int64_t* thr_idx;
  int64_t* left;
  unsigned long long* acount;
  int64_t* aptr;
  int64_t* arank;
  uint64_t* athr_key;
  int64_t* athr_idx;
};

size_t bounded_reserve(Work& w, int64_t n, int32_t k, std::vector<size_t>& o) {
  o.clear();
  o.push_back(w.take(4 * (size_t)n));      // tgt
  o.push_back(w.take(8 * (size_t)n));      // key
  o.push_back(w.take(8 * (size_t)n));      // skey
  o.push_back(w.take(8 * (size_t)n));      // sidx
  o.push_back(w.take(8 * (size_t)n));      // akey
  o.push_back(w.take(8 * (size_t)n));      // aidx
  o.push_back(w.take(8 * (size_t)k));      // cnt
  o.push_back(w.take(8 * (size_t)k));      // pcnt
  o.push_back(w.take(8 * (size_t)k));      // cursor
  o.push_back(w.take(8 * (size_t)k + 8));  // seg_ptr
  o.push_back(w.take(8 * (size_t)k));      // rank
  o.push_back(w.take(8 * (size_t)k));      // thr_key
  o.push_back(w.take(8 * (size_t)k));      // thr_idx
  o.push_back(w.take(64));                 // left, acount, aptr[2], arank, athr_key, athr_idx
  return o.size();
}

BoundedWs bounded_ws(Work& w, const std::vector<size_t>& o) {
  BoundedWs b;
  b.tgt = w.at<int32_t>(o[0]);
  b.key = w.at<double>(o[1]);
  b.skey = w.at<uint64_t>(o[2]);
  b.sidx = w.at<int64_t>(o[3]);
  b.akey = w.at<uint64_t>(o[4]);
  b.aidx = w.at<int64_t>(o[5]);
  b.cnt = w.at<int64_t>(o[6]);
  b.pcnt = w.at<unsigned long long>(o[7]);
  b.cursor = w.at<unsigned long long>(o[8]);
  b.seg_ptr = w.at<int64_t>(o[9]);
  b.rank = w.at<int64_t>(o[10]);
  b.thr_key = w.at<uint64_t>(o[11]);
  b.thr_idx = w.at<int64_t>(o[12]);
  char* s = w.at<char>(o[13]);
  b.left = reinterpret_cast<int64_t*>(s);
  b.acount = reinterpret_cast<unsigned long long*>(s + 8);
  b.aptr = reinterpret_cast<int64_t*>(s + 16);
  b.arank = reinterpret_cast<int64_t*>(s + 32);
  b.athr_key = reinterpret_cast<uint64_t*>(s + 40);
  b.athr_idx = reinterpret_cast<int64_t*>(s + 48);
  return b;
}

// Capacity-bounded assignment into label (device [n]); counts stay in b.cnt.
int32_t bounded(const double* P, int64_t n, int32_t d, const double* C, int32_t k, int64_t lo, int64_t hi,
                int32_t* label, const BoundedWs& b, hipStream_t st) {
  const int64_t nb = nblocks(n);
  // label = -1, counts and proposal counts 0, n points left
  HIPCHK(hipMemsetAsync(label, 0xff, 4 * (size_t)n, st));
  HIPCHK(hipMemsetAsync(b.cnt, 0, 8 * (size_t)k, st));
  HIPCHK(hipMemsetAsync(b.pcnt, 0, 8 * (size_t)k, st));
  HIPCHK(hipMemsetAsync(b.acount, 0, 8, st));
  HIPCHK(hipMemcpyAsync(b.left, &n, 8, hipMemcpyHostToDevice, st));
  int32_t rounds = 0;
  int64_t left = n;
  while (left > 0) {
    if (rounds > k + 1) throw Err{LMA_E_INTERNAL, "bounded assignment did not finish in k + 1 rounds"};
    ++rounds;
    hipLaunchKernelGGL(k_propose, dim3((unsigned)nb), dim3(NT), 0, st, P, n, (int)d, C, (int)k, hi, b.cnt, label,
                       b.tgt, b.key, b.pcnt);
    chk();
    hipLaunchKernelGGL(k_seg_offsets, dim3(1), dim3(1024), 0, st, b.pcnt, (int)k, b.seg_ptr, b.cursor, b.cnt, hi, 0,
                       b.rank);
    chk();
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)nb), dim3(NT), 0, st, n, label, 0, b.tgt, b.key, b.seg_ptr,
                       b.cursor, b.skey, b.sidx);
    chk();
    hipLaunchKernelGGL(k_seg_select, dim3((unsigned)k), dim3(NT), 0, st, b.seg_ptr, b.skey, b.sidx, b.rank, (int)k,
                       b.thr_key, b.thr_idx);
    chk();
    hipLaunchKernelGGL(k_accept, dim3((unsigned)nb), dim3(NT), 0, st, n, label, b.tgt, b.key, b.thr_key, b.thr_idx);
    chk();
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(1024), 0, st, (int)k, b.seg_ptr, hi, b.cnt, b.left);
    chk();
    HIPCHK(hipMemcpyAsync(&left, b.left, 8, hipMemcpyDeviceToHost, st));
    sync(st);
  }
  if (lo <= 0) return rounds;
  std::vector<int64_t> cnt(k);
  HIPCHK(hipMemcpyAsync(cnt.data(), b.cnt, 8 * (size_t)k, hipMemcpyDeviceToHost, st));
  sync(st);
  for (int c = 0; c < k; ++c) {
    if (cnt[c] >= lo) continue;
    hipLaunchKernelGGL(k_lb_keys, dim3((unsigned)nb), dim3(NT), 0, st, P, n, (int)d, C, c, label, b.cnt, lo, b.tgt,
                       b.key, b.pcnt);
    chk();
    hipLaunchKernelGGL(k_seg_offsets, dim3(1), dim3(1024), 0, st, b.pcnt, (int)k, b.seg_ptr, b.cursor, b.cnt, lo, 1,
                       b.rank);
    chk();
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)nb), dim3(NT), 0, st, n, label, 1, b.tgt, b.key, b.seg_ptr,
                       b.cursor, b.skey, b.sidx);
    chk();
    hipLaunchKernelGGL(k_seg_select, dim3((unsigned)k), dim3(NT), 0, st, b.seg_ptr, b.skey, b.sidx, b.rank, (int)k,
                       b.thr_key, b.thr_idx);
    chk();
    hipLaunchKernelGGL(k_lb_gather, dim3((unsigned)nb), dim3(NT), 0, st, n, b.tgt, b.key, b.thr_key, b.thr_idx,
                       b.akey, b.aidx, b.acount);
    chk();
    hipLaunchKernelGGL(k_lb_seg, dim3(1), dim3(1), 0, st, b.acount, b.cnt, c, lo, b.aptr, b.arank);
    chk();
    hipLaunchKernelGGL(k_seg_select, dim3(1), dim3(NT), 0, st, b.aptr, b.akey, b.aidx, b.arank, 1, b.athr_key,
                       b.athr_idx);
    chk();
    hipLaunchKernelGGL(k_lb_move, dim3((unsigned)nb), dim3(NT), 0, st, n, c, label, b.tgt, b.key, b.thr_key,
                       b.thr_idx, b.athr_key, b.athr_idx, reinterpret_cast<unsigned long long*>(b.cnt));
    chk();
    hipLaunchKernelGGL(k_lb_fix, dim3(1), dim3(1), 0, st, b.cnt, c, lo, b.acount);
    chk();
  }
  return rounds;
}

void check_bounds(int64_t n, int32_t k, int64_t lo, int64_t hi) {
  if (hi < 1 || lo < 0 || lo > hi) throw Err{LMA_E_ARG, "need 0 <= lo <= hi and hi >= 1"};
  if ((int64_t)k * lo > n || (int64_t)k * hi < n)
    throw Err{LMA_E_ARG, "block size bounds cannot be met: need k*lo <= n <= k*hi"};
}

// Stable sort of keys [n] (each < nkeys) carrying the point index: perm [n].
void stable_perm(const uint32_t* keys, int64_t n, int64_t nkeys, int64_t* perm, uint32_t* kbuf, int64_t* vbuf,
                 uint32_t* H, hipStream_t st) {
  if (n == 0) return;
  const int64_t nch = (n + SORT_CHUNK - 1) / SORT_CHUNK;
  const int passes = nkeys <= 256 ? 1 : 2;
  const uint32_t* kin = keys;
  const int64_t* vin = nullptr;
  for (int ps = 0; ps < passes; ++ps) {
    const bool last = ps == passes - 1;
    uint32_t* kout = kbuf + (ps & 1) * n;
    int64_t* vout = last ? perm : vbuf + (ps & 1) * n;
    hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)nch), dim3(NT), 0, st, kin, n, 8 * ps, nch, H);
    chk();
    hipLaunchKernelGGL(k_hist_scan, dim3(1), dim3(1024), 0, st, H, 256 * nch);
    chk();
    hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)nch), dim3(NT), 0, st, kin, vin, n, 8 * ps, nch, H, kout,
                       vout);
    chk();
    kin = kout;
    vin = vout;
  }
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

lma_status lma_kmeans_seed(const double* P, int64_t n, int32_t d, int32_t k, const uint32_t* rand, double* C,
                           int64_t* index, hipStream_t stream) {
  return guard([&] {
    check_pts(P, n, d, "P");
    if (n < 1) throw Err{LMA_E_ARG, "need n >= 1"};
    if (k < 1 || k > MAX_K) throw Err{LMA_E_ARG, "need 1 <= k <= 65536"};
    if (!rand || !C) throw Err{LMA_E_ARG, "NULL array"};
    const int64_t nb = nblocks(n);
    Work w;
    const size_t o_dmin = w.take(8 * (size_t)n), o_bmax = w.take(8 * (size_t)nb), o_bsum = w.take(8 * (size_t)nb);
    const size_t o_scal = w.take(16), o_rnd = w.take(4 * (size_t)k), o_sidx = w.take(8 * (size_t)k);
    w.get(stream);
    check_finite(P, n * d, w.at<int32_t>(o_scal), stream, "P");
    int64_t* sidx = index ? index : w.at<int64_t>(o_sidx);
    seed(P, n, d, k, rand, C, sidx, w.at<double>(o_dmin), w.at<double>(o_bmax), w.at<uint64_t>(o_bsum),
         w.at<int32_t>(o_scal), w.at<uint32_t>(o_rnd), stream);
  });
}

lma_status lma_bounded_assign(const double* P, int64_t n, int32_t d, const double* C, int32_t k, int64_t lo,
                              int64_t hi, int32_t* label, int64_t* count, int32_t* rounds, hipStream_t stream) {
  return guard([&] {
    check_pts(P, n, d, "P");
    if (k < 1 || k > MAX_K) throw Err{LMA_E_ARG, "need 1 <= k <= 65536"};
    if (!C || (n > 0 && !label)) throw Err{LMA_E_ARG, "NULL array"};
    check_bounds(n, k, lo, hi);
    Work w;
    std::vector<size_t> o;
    bounded_reserve(w, n, k, o);
    const size_t o_flag = w.take(16);
    w.get(stream);
    check_finite(P, n * d, w.at<int32_t>(o_flag), stream, "P");
    check_finite(C, (int64_t)k * d, w.at<int32_t>(o_flag), stream, "C");
    const BoundedWs b = bounded_ws(w, o);
    int32_t r = 0;
    if (n > 0) r = bounded(P, n, d, C, k, lo, hi, label, b, stream);
    else HIPCHK(hipMemsetAsync(b.cnt, 0, 8 * (size_t)k, stream));
    if (count) HIPCHK(hipMemcpyAsync(count, b.cnt, 8 * (size_t)k, hipMemcpyDeviceToDevice, stream));
    if (rounds) *rounds = r;
    sync(stream);
  });
}

lma_status lma_partition(const double* X, int64_t n, const double* U, int64_t n_u, int32_t d, int32_t M, int64_t lo,
                         int64_t hi, int32_t iters, const uint32_t* rand, int64_t* perm, int64_t* block_ptr,
                         int64_t* u_perm, int64_t* u_block_ptr, double* centres, hipStream_t stream) {
  return guard([&] {
    check_pts(X, n, d, "X");
    check_pts(U, n_u, d, "U");
    if (n < 1) throw Err{LMA_E_ARG, "need n >= 1"};
    if (M < 1 || M > MAX_K) throw Err{LMA_E_ARG, "need 1 <= M <= 65536"};
    if (iters < 0) throw Err{LMA_E_ARG, "iters < 0"};
    if (!rand || !perm || !block_ptr) throw Err{LMA_E_ARG, "NULL array"};
    if (n_u > 0 && (!u_perm || !u_block_ptr)) throw Err{LMA_E_ARG, "NULL test-point output"};
    check_bounds(n, M, lo, hi);
    const int64_t nb = nblocks(n), nmax = std::max(n, n_u);
    const int64_t nch = (nmax + SORT_CHUNK - 1) / SORT_CHUNK;
    Work w;
    std::vector<size_t> o;
    bounded_reserve(w, n, M, o);
    const size_t o_dmin = w.take(8 * (size_t)n), o_bmax = w.take(8 * (size_t)nb), o_bsum = w.take(8 * (size_t)nb);
    const size_t o_scal = w.take(16), o_rnd = w.take(4 * (size_t)M), o_sidx = w.take(8 * (size_t)M);
    const size_t o_C = w.take(8 * (size_t)M * d), o_Cb = w.take(8 * (size_t)M * d);
    const size_t o_label = w.take(4 * (size_t)nmax), o_keys = w.take(4 * (size_t)nmax);
    const size_t o_kbuf = w.take(8 * (size_t)nmax), o_vbuf = w.take(16 * (size_t)nmax);
    const size_t o_H = w.take(4 * 256 * (size_t)nch), o_rank = w.take(4 * (size_t)M);
    const size_t o_bc = w.take(8 * (size_t)M), o_dist = w.take(8 * (size_t)nmax);
    w.get(stream);
    int32_t* flag = w.at<int32_t>(o_scal);
    check_finite(X, n * d, flag, stream, "X");
    check_finite(U, n_u * d, flag, stream, "U");
    double* C = w.at<double>(o_C);
    int32_t* label = w.at<int32_t>(o_label);
    // 1. seeding, 2. Lloyd
    seed(X, n, d, M, rand, C, w.at<int64_t>(o_sidx), w.at<double>(o_dmin), w.at<double>(o_bmax),
         w.at<uint64_t>(o_bsum), w.at<int32_t>(o_scal), w.at<uint32_t>(o_rnd), stream);
    {
      const lma_status s = lma_kmeans(X, n, d, C, M, iters, label, w.at<double>(o_dist), stream);
      if (s != LMA_OK) throw Err{s, std::string("Lloyd: ") + lma_last_error()};
    }
    // 3. bounded assignment, 4. block centres
    const BoundedWs b = bounded_ws(w, o);
    bounded(X, n, d, C, M, lo, hi, label, b, stream);
    double* Cb = w.at<double>(o_Cb);
    HIPCHK(hipMemcpyAsync(Cb, C, 8 * (size_t)M * d, hipMemcpyDeviceToDevice, stream));
    {
      const lma_status s = lma_kmeans_update(X, n, d, label, M, Cb, nullptr, stream);
      if (s != LMA_OK) throw Err{s, std::string("block centres: ") + lma_last_error()};
    }
    // 5. chain order of the block centres (host)
    std::vector<double> Ch((size_t)M * d);
    HIPCHK(hipMemcpyAsync(Ch.data(), Cb, 8 * (size_t)M * d, hipMemcpyDeviceToHost, stream));
    sync(stream);
    std::vector<int32_t> chain(M), rank(M);
    {
      const lma_status s = lma_chain_order(Ch.data(), M, d, chain.data());
      if (s != LMA_OK) throw Err{s, std::string("chain order: ") + lma_last_error()};
    }
    for (int m = 0; m < M; ++m) rank[chain[m]] = m;
    int32_t* rank_d = w.at<int32_t>(o_rank);
    HIPCHK(hipMemcpyAsync(rank_d, rank.data(), 4 * (size_t)M, hipMemcpyHostToDevice, stream));
    std::vector<double> Co;  // host source of an asynchronous copy: lives until the final synchronisation
    if (centres) {
      Co.resize((size_t)M * d);
      for (int m = 0; m < M; ++m)
        std::copy(Ch.begin() + (size_t)chain[m] * d, Ch.begin() + (size_t)(chain[m] + 1) * d, Co.begin() + (size_t)m * d);
      HIPCHK(hipMemcpyAsync(centres, Co.data(), 8 * (size_t)M * d, hipMemcpyHostToDevice, stream));
    }
    // 6-7. block keys, stable permutations, block pointers (training, then test)
    uint32_t* keys = w.at<uint32_t>(o_keys);
    unsigned long long* bc = w.at<unsigned long long>(o_bc);
    std::vector<int64_t> cnt(M);
    auto one_set = [&](const int32_t* lab, int64_t np, int64_t* out_perm, int64_t* out_ptr) {
      HIPCHK(hipMemsetAsync(bc, 0, 8 * (size_t)M, stream));
      if (np > 0) {
        hipLaunchKernelGGL(k_block_keys, dim3((unsigned)nblocks(np)), dim3(NT), 0, stream, lab, rank_d, np, keys, bc);
        chk();
        stable_perm(keys, np, M, out_perm, w.at<uint32_t>(o_kbuf), w.at<int64_t>(o_vbuf), w.at<uint32_t>(o_H),
                    stream);
      }
      HIPCHK(hipMemcpyAsync(cnt.data(), bc, 8 * (size_t)M, hipMemcpyDeviceToHost, stream));
      sync(stream);
      out_ptr[0] = 0;
      for (int m = 0; m < M; ++m) out_ptr[m + 1] = out_ptr[m] + cnt[m];
    };
    one_set(label, n, perm, block_ptr);
    if (n_u > 0) {
      // 6. test points to the nearest block centre (unbounded)
      const lma_status s = lma_kmeans_assign(U, n_u, d, Cb, M, label, nullptr, stream);
      if (s != LMA_OK) throw Err{s, std::string("test assignment: ") + lma_last_error()};
      one_set(label, n_u, u_perm, u_block_ptr);
    } else if (u_block_ptr) {
      for (int m = 0; m <= M; ++m) u_block_ptr[m] = 0;
    }
  });
}

}  // extern "C"
