// k-means steps of the block partitioner on gfx950 (include/lma_part.h).
//
// Nearest-centre assignment: one thread per point.  The centres are read with
// wave-uniform loads (every lane of a wave reads the same centre entry), eight
// centres per pass, so a lane keeps eight running sums in registers and reads
// each of its point's coordinates once per pass.  Each distance is summed over
// the coordinates in increasing order with separately rounded products and
// sums (contraction into fused multiply-adds is switched off), so the result
// is the same bit for bit as any plain evaluation in that order.
//
// Centre update: the points are cut into chunks of 4096 consecutive indices.
// One thread per (chunk, centre, coordinate) walks its chunk in increasing
// index and adds the coordinate of the points with its label (the label read
// is wave-uniform); a second kernel adds the chunk sums in chunk order and
// divides once by the count.  Every sum has a fixed order, so the update does
// not depend on scheduling, and the walk spreads over chunks x centres x
// coordinates threads (10752 waves at n=524288, k=256, d=21).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "lma_part.h"
#include "misc.h"
#include "runtime.h"

namespace lma {
namespace part {

constexpr int NTA = 256;   // threads per workgroup, assignment
constexpr int CG = 8;      // centres per pass
constexpr int NTU = 64;    // threads per workgroup, update
constexpr int MAX_K = 65536;
constexpr int64_t CHUNK = 4096;         // points per partial sum of the update
constexpr int64_t PART_BYTES = 1ll << 30;  // partial sums held at once

// Scratch of the allocation-free centre update (lma_kmeans_update_noalloc):
// one copy per GPU, held until the process ends.  Host code never passes the
// symbol itself to a kernel (on the host it is only a stand-in); it uses the
// device address that hipGetSymbolAddress returns for the current device.
constexpr int64_t NOALLOC_BYTES = 16ll << 20;
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

__global__ __launch_bounds__(NTA) void k_km_assign(const double* __restrict__ P, int64_t n, int d,
                                                   const double* __restrict__ C, int k, int32_t* __restrict__ label,
                                                   double* __restrict__ dist2) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * NTA + threadIdx.x;
  if (i >= n) return;
  const double* p = P + i * d;
  double best = INFINITY;
  int arg = 0;
  for (int c0 = 0; c0 < k; c0 += CG) {
    const int nc = k - c0 < CG ? k - c0 : CG;
    double acc[CG];
#pragma unroll
    for (int j = 0; j < CG; ++j) acc[j] = 0.0;
    const double* cb = C + (int64_t)c0 * d;
    for (int t = 0; t < d; ++t) {
      const double x = p[t];
#pragma unroll
      for (int j = 0; j < CG; ++j) {
        if (j < nc) {
          const double df = x - cb[j * d + t];
          const double sq = df * df;
          acc[j] = acc[j] + sq;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < CG; ++j)
      if (j < nc && acc[j] < best) {
        best = acc[j];
        arg = c0 + j;
      }
  }
  label[i] = arg;
  if (dist2) dist2[i] = best;
}

__global__ __launch_bounds__(NTU) void k_km_partial(const double* __restrict__ P, int64_t n, int d,
                                                    const int32_t* __restrict__ label, int k, int64_t ch0,
                                                    int64_t nbx, double* __restrict__ part,
                                                    int64_t* __restrict__ pcnt) {
  // block b covers chunk ch0 + b / nbx and threads (b % nbx) * NTU + tid of the k*d (centre, coordinate) pairs
  const int64_t kd = (int64_t)k * d;
  const int64_t g = blockIdx.x / nbx;
  const int64_t e = (blockIdx.x - g * nbx) * NTU + threadIdx.x;
  if (e >= kd) return;
  const int c = (int)(e / d), t = (int)(e - (int64_t)c * d);
  const int64_t i0 = (ch0 + g) * CHUNK;
  const int64_t i1 = i0 + CHUNK < n ? i0 + CHUNK : n;
  double s = 0.0;
  int64_t cnt = 0;
  int64_t i = i0;
  for (; i + 8 <= i1; i += 8) {
    int32_t lb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) lb[j] = label[i + j];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (lb[j] == c) {
        s = s + P[(i + j) * d + t];
        ++cnt;
      }
  }
  for (; i < i1; ++i)
    if (label[i] == c) {
      s = s + P[i * d + t];
      ++cnt;
    }
  part[g * kd + e] = s;
  if (t == 0) pcnt[g * k + c] = cnt;
}

__global__ __launch_bounds__(NTU) void k_km_combine(const double* __restrict__ part, const int64_t* __restrict__ pcnt,
                                                    int64_t nch, int k, int d, double* __restrict__ srun,
                                                    int64_t* __restrict__ crun, int first, int last,
                                                    double* __restrict__ C, int64_t* __restrict__ count) {
  const int64_t kd = (int64_t)k * d;
  const int64_t e = (int64_t)blockIdx.x * NTU + threadIdx.x;
  if (e >= kd) return;
  const int c = (int)(e / d), t = (int)(e - (int64_t)c * d);
  double s = first ? 0.0 : srun[e];
  int64_t cnt = first ? 0 : crun[e];
  for (int64_t g = 0; g < nch; ++g) {
    s = s + part[g * kd + e];
    cnt += pcnt[g * k + c];
  }
  if (!last) {
    srun[e] = s;
    crun[e] = cnt;
    return;
  }
  if (cnt > 0) C[e] = s / (double)cnt;
  if (count && t == 0) count[c] = cnt;
}

}  // namespace part
}  // namespace lma

namespace {

using lmart::Err;

void check_shape(const double* P, int64_t n, int32_t d, int32_t k) {
  if (n < 0) throw Err{LMA_E_ARG, "n < 0"};
  if (d < 1 || d > lma::MAX_D) throw Err{LMA_E_ARG, "need 1 <= d <= 64"};
  if (k < 1 || k > lma::part::MAX_K) throw Err{LMA_E_ARG, "need 1 <= k <= 65536"};
  if (n > 0 && !P) throw Err{LMA_E_ARG, "P is NULL"};
}

void assign(const double* P, int64_t n, int32_t d, const double* C, int32_t k, int32_t* label, double* dist2,
            hipStream_t st) {
  if (n == 0) return;
  const int64_t nb = (n + lma::part::NTA - 1) / lma::part::NTA;
  if (nb > 0x7fffffff) throw Err{LMA_E_ARG, "too many points"};
  hipLaunchKernelGGL(lma::part::k_km_assign, dim3((unsigned)nb), dim3(lma::part::NTA), 0, st, P, n, (int)d, C, (int)k,
                     label, dist2);
  HIPCHK(hipGetLastError());
}

// Centre update in chunk order.  Chunks are processed in groups of `group`
// chunks whose partial sums sit at the start of the workspace `mem`; running
// sums (after them) carry the order across groups, so the result does not
// depend on the group size.  Returns the launch status; enqueues only.
hipError_t update_launch(const double* P, int64_t n, int32_t d, const int32_t* label, int32_t k, double* C,
                         int64_t* count, int64_t group, char* mem, hipStream_t st) {
  using namespace lma::part;
  const int64_t kd = (int64_t)k * d;
  const int64_t nch = n > 0 ? (n + CHUNK - 1) / CHUNK : 0;
  const int64_t per = (int64_t)sizeof(double) * kd + (int64_t)sizeof(int64_t) * k;
  const int64_t nbx = (kd + NTU - 1) / NTU;
  double* part = reinterpret_cast<double*>(mem);
  int64_t* pcnt = reinterpret_cast<int64_t*>(mem + sizeof(double) * group * kd);
  double* srun = reinterpret_cast<double*>(mem + group * per);
  int64_t* crun = reinterpret_cast<int64_t*>(mem + group * per + sizeof(double) * kd);
  hipError_t err = hipSuccess;
  if (nch == 0) {
    hipLaunchKernelGGL(k_km_combine, dim3((unsigned)nbx), dim3(NTU), 0, st, part, pcnt, (int64_t)0, (int)k, (int)d,
                       srun, crun, 1, 1, C, count);
    err = hipGetLastError();
  }
  for (int64_t ch0 = 0; ch0 < nch && err == hipSuccess; ch0 += group) {
    const int64_t ng = std::min<int64_t>(group, nch - ch0);
    hipLaunchKernelGGL(k_km_partial, dim3((unsigned)(ng * nbx)), dim3(NTU), 0, st, P, n, (int)d, label, (int)k, ch0,
                       nbx, part, pcnt);
    err = hipGetLastError();
    if (err != hipSuccess) break;
    hipLaunchKernelGGL(k_km_combine, dim3((unsigned)nbx), dim3(NTU), 0, st, part, pcnt, ng, (int)k, (int)d, srun,
                       crun, ch0 == 0 ? 1 : 0, ch0 + ng >= nch ? 1 : 0, C, count);
    err = hipGetLastError();
  }
  return err;
}

// Bytes of partial sums per chunk, and of the running sums.
int64_t update_per_chunk(int32_t d, int32_t k) {
  return (int64_t)sizeof(double) * k * d + (int64_t)sizeof(int64_t) * k;
}
int64_t update_running(int32_t d, int32_t k) {
  return (int64_t)(sizeof(double) + sizeof(int64_t)) * k * d;
}

void check_launch_size(int64_t group, int32_t d, int32_t k) {
  const int64_t nbx = ((int64_t)k * d + lma::part::NTU - 1) / lma::part::NTU;
  if (group * nbx > 0x7fffffff) throw Err{LMA_E_ARG, "too many centres x coordinates for one launch"};
}

// The update with a workspace from the library's device cache (partial sums
// of at most PART_BYTES at once), returned after a stream synchronisation.
void update(const double* P, int64_t n, int32_t d, const int32_t* label, int32_t k, double* C, int64_t* count,
            hipStream_t st) {
  using namespace lma::part;
  const int64_t nch = n > 0 ? (n + CHUNK - 1) / CHUNK : 0;
  const int64_t per = update_per_chunk(d, k);
  int64_t cap = PART_BYTES;
  if (const char* env = std::getenv("LMA_KMEANS_PART_BYTES")) cap = std::max<long long>(1, std::atoll(env));
  const int64_t group = nch == 0 ? 0 : std::max<int64_t>(1, std::min<int64_t>(nch, cap / per));
  check_launch_size(group, d, k);
  const size_t bytes = (size_t)(group * per + update_running(d, k));
  char* mem = static_cast<char*>(lmart::devcache::get(bytes));
  if (!mem) throw Err{LMA_E_NOMEM, "device allocation for the centre update failed"};
  const hipError_t err = update_launch(P, n, d, label, k, C, count, group, mem, st);
  const hipError_t es = hipStreamSynchronize(st);
  lmart::devcache::put(mem, bytes);
  if (err != hipSuccess) throw Err{LMA_E_HIP, std::string("k-means update launch: ") + hipGetErrorString(err)};
  if (es != hipSuccess) throw Err{LMA_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(es)};
}

// Device address of the scratch array on the current device, looked up once
// per device (each GPU holds its own copy at its own address).
char* scratch_ptr() {
  static std::mutex mu;
  static std::vector<char*> ptrs;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
  if (!ptrs[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(lma::part::scratch));
    if (e != hipSuccess || !ptr)
      throw Err{LMA_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    ptrs[dev] = static_cast<char*>(ptr);
  }
  return ptrs[dev];
}

// The update in the fixed scratch array: no allocation and no synchronisation.
void update_noalloc(const double* P, int64_t n, int32_t d, const int32_t* label, int32_t k, double* C,
                    int64_t* count, hipStream_t st) {
  using namespace lma::part;
  const int64_t nch = n > 0 ? (n + CHUNK - 1) / CHUNK : 0;
  const int64_t per = update_per_chunk(d, k);
  const int64_t room = NOALLOC_BYTES - update_running(d, k);
  if (room < per)
    throw Err{LMA_E_ARG, "k * d too large for the allocation-free update: need 24 k d + 8 k <= " +
                             std::to_string(NOALLOC_BYTES) + " bytes"};
  const int64_t group = nch == 0 ? 0 : std::max<int64_t>(1, std::min<int64_t>(nch, room / per));
  check_launch_size(group, d, k);
  char* mem = scratch_ptr();
  const hipError_t err = update_launch(P, n, d, label, k, C, count, group, mem, st);
  if (err != hipSuccess) throw Err{LMA_E_HIP, std::string("k-means update launch: ") + hipGetErrorString(err)};
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

#pragma clang fp contract(off)
double host_sqdist(const double* a, const double* b, int d) {
  double acc = 0.0;
  for (int t = 0; t < d; ++t) {
    const double df = a[t] - b[t];
    const double sq = df * df;
    acc = acc + sq;
  }
  return acc;
}

void chain_order(const double* C, int k, int d, int32_t* order) {
  std::vector<double> mean(d, 0.0);
  for (int c = 0; c < k; ++c)
    for (int t = 0; t < d; ++t) mean[t] = mean[t] + C[(int64_t)c * d + t];
  for (int t = 0; t < d; ++t) mean[t] = mean[t] / (double)k;
  int cur = 0;
  double far = -1.0;
  for (int c = 0; c < k; ++c) {
    const double q = host_sqdist(C + (int64_t)c * d, mean.data(), d);
    if (q > far) {
      far = q;
      cur = c;
    }
  }
  std::vector<char> seen(k, 0);
  order[0] = cur;
  seen[cur] = 1;
  for (int step = 1; step < k; ++step) {
    int nxt = -1;
    double best = 0.0;
    for (int c = 0; c < k; ++c) {
      if (seen[c]) continue;
      const double q = host_sqdist(C + (int64_t)c * d, C + (int64_t)cur * d, d);
      if (nxt < 0 || q < best) {
        best = q;
        nxt = c;
      }
    }
    order[step] = nxt;
    seen[nxt] = 1;
    cur = nxt;
  }
}

}  // namespace

extern "C" {

lma_status lma_kmeans_assign(const double* P, int64_t n, int32_t d, const double* C, int32_t k, int32_t* label,
                             double* dist2, hipStream_t stream) {
  return guard([&] {
    check_shape(P, n, d, k);
    if (n > 0 && (!C || !label)) throw Err{LMA_E_ARG, "NULL array"};
    assign(P, n, d, C, k, label, dist2, stream);
  });
}

lma_status lma_kmeans_update(const double* P, int64_t n, int32_t d, const int32_t* label, int32_t k, double* C,
                             int64_t* count, hipStream_t stream) {
  return guard([&] {
    check_shape(P, n, d, k);
    if (!C || (n > 0 && !label)) throw Err{LMA_E_ARG, "NULL array"};
    update(P, n, d, label, k, C, count, stream);
  });
}

lma_status lma_kmeans_update_noalloc(const double* P, int64_t n, int32_t d, const int32_t* label, int32_t k,
                                     double* C, int64_t* count, hipStream_t stream) {
  return guard([&] {
    check_shape(P, n, d, k);
    if (!C || (n > 0 && !label)) throw Err{LMA_E_ARG, "NULL array"};
    update_noalloc(P, n, d, label, k, C, count, stream);
  });
}

lma_status lma_kmeans(const double* P, int64_t n, int32_t d, double* C, int32_t k, int32_t iters, int32_t* label,
                      double* dist2, hipStream_t stream) {
  return guard([&] {
    check_shape(P, n, d, k);
    if (iters < 0) throw Err{LMA_E_ARG, "iters < 0"};
    if (!C || (n > 0 && !label)) throw Err{LMA_E_ARG, "NULL array"};
    for (int32_t it = 0; it < iters; ++it) {
      assign(P, n, d, C, k, label, nullptr, stream);
      if (n > 0) update(P, n, d, label, k, C, nullptr, stream);
    }
    assign(P, n, d, C, k, label, dist2, stream);
  });
}

lma_status lma_chain_order(const double* C, int32_t k, int32_t d, int32_t* order) {
  return guard([&] {
    if (d < 1 || d > lma::MAX_D) throw Err{LMA_E_ARG, "need 1 <= d <= 64"};
    if (k < 1) throw Err{LMA_E_ARG, "need k >= 1"};
    if (!C || !order) throw Err{LMA_E_ARG, "NULL array"};
    chain_order(C, k, d, order);
  });
}

}  // extern "C"
