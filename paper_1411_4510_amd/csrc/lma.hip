// Host runtime and C ABI of the LMA library (see include/lma.h).
//
// lma_fit, per problem:
//   1. scale inputs by the length-scales, centre y;
//   2. S run (float64): Cholesky of Sigma_SS with the training rows as
//      right-hand sides -> L_SS and V^T = K_DS L_SS^-T (n x sp);
//   3. window run (float64 or float32): for every block m the window
//      J_m = [D^B_m ; D_m] is factored with the support rows K_SJ and the
//      centred outputs c_J as right-hand sides; the residual R_J = Sigma_JJ -
//      V_J^T V_J is generated tile by tile inside the update kernel
//      (Lemma 1 / Definition 1 in whitened form);
//   4. summary GEMM (float64 accumulation) over the D_m columns of every
//      window: Sigma_ddot_SS - Sigma_SS, y_ddot_S, sum |z_m|^2 (Definition 2);
//   5. Sigma_ddot run (float64): Cholesky of Sigma_ddot_SS; one-workgroup
//      solve for g with iterative refinement (Theorem 2).
// lma_predict: S run and window runs in solve-only mode on the test rows,
// per-point sums G_u, l_u, xi_u over the windows q-B..q of the test block,
// Sigma_ddot solve of k_u - G_u, and the combine of Theorem 2.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "grad.h"
#include "runtime.h"

using namespace lma;

namespace {
thread_local std::string g_err;
thread_local int64_t g_failed = -3;  // -3: no block (see lma_failed_block)
}  // namespace

namespace lmart {

// Device blocks released by lma_free / lma_predict / the end of a fit are
// kept (at most four) and reused by the next call that fits in them: a state
// at the n=524288 workload is ~95 GB and mapping it anew each fit costs a few
// hundred milliseconds.  lma_release_cache() returns them to the runtime.
namespace devcache {
struct Block {
  void* p = nullptr;
  size_t bytes = 0;
  int device = -1;
};
std::mutex mu;
constexpr int NSLOT = 4;
Block slots[NSLOT];
// real size of every block handed out (a cached block can be larger than the
// request it served; it returns to the cache with its real size)
std::map<void*, size_t> out_sizes;
// LMA_CACHE_TRACE=1 prints every cache decision with its host time (stderr)
bool trace() {
  static const bool on = std::getenv("LMA_CACHE_TRACE") != nullptr;
  return on;
}
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
void free_all_locked() {
  const double t0 = trace() ? now_s() : 0.0;
  size_t freed = 0;
  for (Block& b : slots) {
    if (b.p) (void)hipFree(b.p);
    freed += b.bytes;
    b = Block{};
  }
  if (trace()) fprintf(stderr, "[devcache] free all: %.2f GB in %.3f s\n", freed / 1e9, now_s() - t0);
}
void* get(size_t bytes) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(mu);
  int best = -1;
  for (int i = 0; i < NSLOT; ++i)
    if (slots[i].p && slots[i].device == dev && slots[i].bytes >= bytes && slots[i].bytes <= 2 * bytes + (64 << 20) &&
        (best < 0 || slots[i].bytes < slots[best].bytes))
      best = i;
  if (best >= 0) {
    void* p = slots[best].p;
    if (trace()) fprintf(stderr, "[devcache] get %.2f GB: cached block of %.2f GB\n", bytes / 1e9, slots[best].bytes / 1e9);
    out_sizes[p] = slots[best].bytes;
    slots[best] = Block{};
    return p;
  }
  const double t0 = trace() ? now_s() : 0.0;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess || !p) {
    (void)hipGetLastError();
    free_all_locked();  // make room, then try once more
    p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  if (trace()) fprintf(stderr, "[devcache] get %.2f GB: hipMalloc in %.3f s\n", bytes / 1e9, now_s() - t0);
  out_sizes[p] = bytes;
  return p;
}
void put(void* p, size_t bytes) {
  if (!p) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(mu);
  const auto known = out_sizes.find(p);
  if (known != out_sizes.end()) {
    bytes = known->second;
    out_sizes.erase(known);
  }
  int victim = 0;
  for (int i = 0; i < NSLOT; ++i)
    if (!slots[i].p) {
      victim = i;
      break;
    } else if (slots[i].bytes < slots[victim].bytes) {
      victim = i;
    }
  if (slots[victim].p) {
    const double t0 = trace() ? now_s() : 0.0;
    (void)hipFree(slots[victim].p);
    if (trace()) fprintf(stderr, "[devcache] evict %.2f GB in %.3f s\n", slots[victim].bytes / 1e9, now_s() - t0);
  }
  if (trace()) fprintf(stderr, "[devcache] put %.2f GB\n", bytes / 1e9);
  slots[victim] = Block{p, bytes, dev};
}
void release() {
  std::lock_guard<std::mutex> lk(mu);
  free_all_locked();
}
}  // namespace devcache

void set_last_error(const std::string& msg) { g_err = msg; }

bool g_inited = false;
void ensure_init() {
  if (g_inited) return;
  HIPCHK(engine_init());
  HIPCHK(misc_init());
  HIPCHK(vecsolve_init());
  HIPCHK(grad_init());
  HIPCHK(kvec_init());
  g_inited = true;
}

// ---------------------------------------------------------------------------
// live timing: HIP events around launches (enabled by lma_profile_enable)
// ---------------------------------------------------------------------------
namespace prof {
bool on = false;
std::vector<Rec> pending;
std::vector<hipEvent_t> pool;
lma_profile acc = {};
hipEvent_t get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}
// call after the stream has been synchronised
void flush() {
  for (const Rec& r : pending) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    switch (r.kind) {
      case UPDATE:
        acc.update_ms += ms;
        acc.update_alg_flops += r.flops;
        acc.update_alg_flops_f64 += r.flops64;
        acc.update_launches += 1;
        break;
      case DIAG: acc.diag_ms += ms; break;
      case TRSM: acc.trsm_ms += ms; break;
      case GEMM:
        acc.gemm_ms += ms;
        acc.gemm_alg_flops += r.flops;
        acc.gemm_launches += 1;
        break;
      case CONTRACT:
        acc.contract_ms += ms;
        acc.contract_alg_flops += r.flops;
        acc.contract_launches += 1;
        break;
      default:
        acc.other_ms += ms;
        acc.other_launches += 1;
    }
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
}
}  // namespace prof

}  // namespace lmart

using namespace lmart;

namespace {

void check_problem(const lma_problem* p) {
  if (!p) throw Err{LMA_E_ARG, "problem is NULL"};
  if (p->n < 1 || p->d < 1 || p->d > MAX_D || p->s < 1 || p->M < 1 || p->B < 0)
    throw Err{LMA_E_ARG, "need n >= 1, 1 <= d <= 64, s >= 1, M >= 1, B >= 0"};
  if (p->M > p->n) throw Err{LMA_E_ARG, "more blocks than training inputs"};
  if (align_up(p->s, TB) > MAX_SP) throw Err{LMA_E_ARG, "support set larger than 8192"};
  if (!p->X || !p->y || !p->S || !p->block_ptr || !p->log_hyp) throw Err{LMA_E_ARG, "NULL array"};
  if (p->precision != LMA_FP64 && p->precision != LMA_MIXED) throw Err{LMA_E_ARG, "unknown precision"};
  if (p->reserved != 0) throw Err{LMA_E_ARG, "reserved field must be 0"};
  if (p->block_ptr[0] != 0 || p->block_ptr[p->M] != p->n)
    throw Err{LMA_E_ARG, "block_ptr must start at 0 and end at n"};
  for (int64_t m = 0; m < p->M; ++m)
    if (p->block_ptr[m + 1] <= p->block_ptr[m]) throw Err{LMA_E_ARG, "blocks must be non-empty and increasing"};
  for (int64_t t = 0; t < p->d + 2; ++t)
    if (!std::isfinite(p->log_hyp[t])) throw Err{LMA_E_ARG, "non-finite hyperparameter"};
  if (!std::isfinite(p->prior_mean)) throw Err{LMA_E_ARG, "non-finite prior mean"};
}

void set_err(const Err& e) {
  g_err = e.msg;
}

// ---------------------------------------------------------------------------
// fit
// ---------------------------------------------------------------------------
template <typename TW>
void build_window_run(lma_state& f, Run<TW>& run, TW* winbase, const double* Xs, const double* Vt, const TW* c,
                      const double* Ss, bool band, int64_t m0, int64_t m1) {
  const int Ts = (int)f.Ts;
  for (int64_t m = m0; m < m1; ++m) {
    const WinGeom g = win_geom(f.bp, f.M, f.B, m);
    TW* base = winbase + f.win_off[m];
    run.add_problem(g.T, Ts + 1, g.tw, false, (int)m);
    add_window_jtiles<TW>(run.rt, g, base, Xs, Vt, c, f.d, f.sp, band);
    TW* rhs = base + jpanel_off(g.T);
    const int64_t ld = (int64_t)g.T * TB;
    for (int r = 0; r < Ts; ++r) {
      const int nv = (int)std::min<int64_t>(TB, f.s - (int64_t)r * TB);
      const bool f64 = std::is_same<TW, double>::value;
      RowTile<TW> t = make_tile<TW>(rhs + (int64_t)r * TB * ld, ld, nullptr,
                                    f64 ? reinterpret_cast<const TW*>(Ss + (int64_t)r * TB * f.d) : nullptr, nullptr,
                                    nv, TB, SRC_KERNEL, 0);
      t.xs64 = Ss + (int64_t)r * TB * f.d;
      run.rt.push_back(t);
    }
    run.rt.push_back(make_tile<TW>(rhs + (int64_t)Ts * TB * ld, ld, nullptr, nullptr, nullptr, 1, TB, SRC_CVEC, 0));
  }
}

template <typename TW>
void build_summary(lma_state& f, std::vector<GemmTerm<TW>>& terms, TW* winbase) {
  const int Ts = (int)f.Ts;
  const int nt = Ts + 1;
  f.ntile = nt * (nt + 1) / 2;
  f.groups = (int)std::max<int64_t>(1, std::min<int64_t>(f.M, cdiv(1024, f.ntile)));
  const int64_t per = cdiv(f.M, f.groups);
  f.groups = (int)cdiv(f.M, per);
  double* partial = f.ptr<double>(f.o_partial);
  f.sumout.clear();
  terms.clear();
  for (int gi = 0; gi < f.groups; ++gi) {
    const int64_t m0 = gi * per, m1 = std::min<int64_t>(f.M, m0 + per);
    for (int ta = 0; ta < nt; ++ta)
      for (int tb = 0; tb <= ta; ++tb) {
        const int t = ta * (ta + 1) / 2 + tb;
        GemmOut o = gemm_out(partial + ((int64_t)gi * f.ntile + t) * TB * TB, TB, TB, TB, 0, (int)terms.size());
        for (int64_t m = m0; m < m1; ++m) {
          const WinGeom g = win_geom(f.bp, f.M, f.B, m);
          TW* rhs = winbase + f.win_off[m] + jpanel_off(g.T);
          const int64_t ld = (int64_t)g.T * TB;
          GemmTerm<TW> tm;
          tm.a = rhs + (int64_t)ta * TB * ld;
          tm.lda = ld;
          tm.anr = TB;
          tm.b = rhs + (int64_t)tb * TB * ld;
          tm.ldb = ld;
          tm.bnr = TB;
          tm.k0 = g.tw * TB;
          tm.k1 = g.T * TB;
          terms.push_back(tm);
        }
        o.t1 = (int32_t)terms.size();
        f.sumout.push_back(o);
      }
  }
}

// Residual band of one fit: one device block [band | items | row offsets]
// from the device cache, returned when the fit ends, after the stream has
// drained (its kernels may still read it when an error ends the fit early).
struct BandPlan {
  std::vector<BandItem> items;
  std::vector<int64_t> brow;
  int64_t o_items = 0, o_brow = 0, bytes = 0;
  void* mem = nullptr;
  hipStream_t st = nullptr;
  BandPlan() = default;
  BandPlan(const BandPlan&) = delete;
  BandPlan& operator=(const BandPlan&) = delete;
  ~BandPlan() {
    if (mem) {
      (void)hipStreamSynchronize(st);
      devcache::put(mem, (size_t)bytes);
    }
  }
};

// Summary terms of the windows [m0, m1) into group 0, added to what earlier
// chunks left there (chunk order fixes the summation order).
template <typename TW>
void build_summary_chunk(lma_state& f, std::vector<GemmTerm<TW>>& terms, TW* winbase, int64_t m0, int64_t m1,
                         bool accumulate) {
  const int nt = (int)f.Ts + 1;
  f.ntile = nt * (nt + 1) / 2;
  f.groups = 1;
  double* partial = f.ptr<double>(f.o_partial);
  for (int ta = 0; ta < nt; ++ta)
    for (int tb = 0; tb <= ta; ++tb) {
      const int t = ta * (ta + 1) / 2 + tb;
      GemmOut o = gemm_out(partial + (int64_t)t * TB * TB, TB, TB, TB, accumulate ? 1 : 0, (int)terms.size());
      for (int64_t m = m0; m < m1; ++m) {
        const WinGeom g = win_geom(f.bp, f.M, f.B, m);
        TW* rhs = winbase + f.win_off[m] + jpanel_off(g.T);
        const int64_t ld = (int64_t)g.T * TB;
        GemmTerm<TW> tm;
        tm.a = rhs + (int64_t)ta * TB * ld;
        tm.lda = ld;
        tm.anr = TB;
        tm.b = rhs + (int64_t)tb * TB * ld;
        tm.ldb = ld;
        tm.bnr = TB;
        tm.k0 = g.tw * TB;
        tm.k1 = g.T * TB;
        terms.push_back(tm);
      }
      o.t1 = (int32_t)terms.size();
      f.sumout.push_back(o);
    }
}

lma_status do_fit(const lma_problem* p, hipStream_t st, lma_state** out, bool keep) {
  check_problem(p);
  ensure_init();
  std::unique_ptr<lma_state> F(new lma_state());
  lma_state& f = *F;
  f.precision = p->precision;
  f.n = p->n;
  f.d = p->d;
  f.s = p->s;
  f.M = p->M;
  f.B = std::min<int64_t>(p->B, p->M - 1);
  f.sp = align_up(p->s, TB);
  f.Ts = f.sp / TB;
  f.mu = p->prior_mean;
  f.log_hyp.assign(p->log_hyp, p->log_hyp + p->d + 2);
  for (int t = 0; t < MAX_D; ++t) f.ie.v[t] = t < p->d ? std::exp(-p->log_hyp[t]) : 0.0;
  f.sf2 = std::exp(p->log_hyp[p->d]);
  f.sn2 = std::exp(p->log_hyp[p->d + 1]);
  f.bp.assign(p->block_ptr, p->block_ptr + p->M + 1);
  const bool mixed = f.mixed();
  const int64_t n = f.n, d = f.d, s = f.s, sp = f.sp, M = f.M;
  const int Ts = (int)f.Ts;
  const int64_t wsz = mixed ? 4 : 8;

  // ---- window geometry
  f.Tm.resize(M);
  f.twm.resize(M);
  f.win_off.resize(M);
  f.inv_off.resize(M);
  std::vector<int64_t> wel(M), iel(M);
  int maxT = 0;
  for (int64_t m = 0; m < M; ++m) {
    const WinGeom g = win_geom(f.bp, M, f.B, m);
    f.Tm[m] = g.T;
    f.twm[m] = g.tw;
    wel[m] = panel_elems(g.T, Ts + 1);
    iel[m] = (int64_t)g.T * TB * TB;
    maxT = std::max(maxT, g.T);
  }
  f.vec_elems = 0;
  for (int64_t m = 0; m < M; ++m) f.vec_elems += (int64_t)f.Tm[m] * TB;
  // Chunks of consecutive windows whose factors (panels and inverted diagonal
  // tiles) fit in area_cap bytes; area_cap <= 0 puts all windows in one chunk.
  auto set_chunks = [&](int64_t area_cap) -> bool {
    f.chunk.assign(1, 0);
    int64_t wacc = 0, iacc = 0;
    f.win_area = f.inv_area = 0;
    for (int64_t m = 0; m < M; ++m) {
      const int64_t need = wsz * (wel[m] + iel[m]);
      if (area_cap > 0 && need > area_cap) return false;
      if (area_cap > 0 && m > f.chunk.back() && wsz * (wacc + iacc) + need > area_cap) {
        f.chunk.push_back(m);
        wacc = iacc = 0;
      }
      f.win_off[m] = wacc;
      f.inv_off[m] = iacc;
      wacc += wel[m];
      iacc += iel[m];
      f.win_area = std::max(f.win_area, wacc);
      f.inv_area = std::max(f.inv_area, iacc);
    }
    f.chunk.push_back(M);
    return true;
  };
  set_chunks(0);

  // ---- memory plan (redone below with chunks when mem_budget_bytes requires)
  Arena& ar = f.ar;
  auto plan_fixed = [&]() {
    ar = Arena();
    f.o_Xs64 = ar.reserve(8 * n * d);
    f.o_Ss64 = ar.reserve(8 * s * d);
    f.o_c64 = ar.reserve(8 * n);
    if (mixed) f.o_c32 = ar.reserve(4 * n);
    f.o_Vt64 = ar.reserve(8 * n * sp);
    f.o_Lss = ar.reserve(8 * panel_elems(Ts, 0));
    f.o_Lss_inv = ar.reserve(8 * (int64_t)Ts * TB * TB);
    f.o_win = ar.reserve(wsz * f.win_area);
    f.o_win_inv = ar.reserve(wsz * f.inv_area);
    {
      const int nt = Ts + 1, ntile = nt * (nt + 1) / 2;
      int groups = (int)std::max<int64_t>(1, std::min<int64_t>(M, cdiv(1024, ntile)));
      groups = (int)cdiv(M, cdiv(M, groups));
      if (f.streaming()) groups = 1;
      f.o_partial = ar.reserve(8 * (int64_t)groups * ntile * TB * TB);
    }
    f.o_Sdd = ar.reserve(8 * sp * sp);
    f.o_ydd = ar.reserve(8 * sp);
    f.o_q = ar.reserve(8);
    f.o_Ldd = ar.reserve(8 * panel_elems(Ts, 0));
    f.o_Ldd_inv = ar.reserve(8 * (int64_t)Ts * TB * TB);
    f.o_g = ar.reserve(8 * sp);
    f.n_logdiag = (int64_t)(M + 2) * std::max(maxT, Ts);
    f.o_logdiag = ar.reserve(8 * f.n_logdiag);
    f.n_status = M + 2;
    f.o_status = ar.reserve(4 * f.n_status);
    f.o_wt = ar.reserve(8 * 10 * M);
    f.o_xJ = ar.reserve(8 * f.vec_elems);
    f.o_xW = ar.reserve(8 * f.vec_elems);
    f.o_tJ = ar.reserve(8 * f.vec_elems);
    f.o_tW = ar.reserve(8 * f.vec_elems);
    f.o_hJ = ar.reserve(8 * M * sp);
    f.o_hW = ar.reserve(8 * M * sp);
    if (mixed) {
      f.o_cg = ar.reserve(8 * n);
      f.o_dg = ar.reserve(8 * sp);
      f.o_tvec = ar.reserve(8 * sp);
      f.o_rho = ar.reserve(8 * sp);
    }
  };
  plan_fixed();

  // ---- residual band (overlapping windows only): panel of block a spans the
  // points of blocks max(0, a-B) .. a; tiles entirely right of the diagonal
  // are never read and not formed
  BandPlan bpl;
  bool use_band = f.B >= 1 && std::getenv("LMA_NO_BAND") == nullptr;
  if (use_band) {
    bpl.brow.resize(n);
    int64_t off = 0;
    for (int64_t a = 0; a < M; ++a) {
      const int64_t c0 = f.bp[std::max<int64_t>(0, a - f.B)], r0 = f.bp[a], r1 = f.bp[a + 1], w = r1 - c0;
      for (int64_t p = r0; p < r1; ++p) bpl.brow[p] = off + (p - r0) * w - c0;
      // groups of 4 row tiles sweep the column tiles together, so the
      // workgroups running at one time share their V rows in L2
      for (int64_t g0 = r0; g0 < r1; g0 += 4 * TB) {
        const int64_t g1 = std::min<int64_t>(r1, g0 + 4 * TB);
        for (int64_t q0 = c0; q0 < g1; q0 += TB)
          for (int64_t p0 = g0; p0 < g1; p0 += TB) {
            const int nr = (int)std::min<int64_t>(TB, r1 - p0);
            if (q0 > p0 + nr - 1) continue;  // right of the diagonal: never read
            BandItem it;
            it.p0 = p0;
            it.q0 = q0;
            it.off = off + (p0 - r0) * w + (q0 - c0);
            it.ld = w;
            it.nr = nr;
            it.nc = (int)std::min<int64_t>(TB, r1 - q0);
            bpl.items.push_back(it);
          }
      }
      off += (r1 - r0) * w;
    }
    bpl.o_items = align_up(wsz * off, 256);
    bpl.o_brow = bpl.o_items + align_up((int64_t)sizeof(BandItem) * (int64_t)bpl.items.size(), 256);
    bpl.bytes = bpl.o_brow + 8 * n;
  }

  // engine runs (built with arena offsets; pointers fixed after allocation)
  // Reserve space for run metadata: build runs against a null base first to size them.
  auto build_runs = [&](char* base) {
    f.ar.base = base;
    f.runS = Run<double>();
    f.runD = Run<double>();
    const int nch = (int)f.chunk.size() - 1;
    f.runsW32.assign(mixed ? nch : 0, Run<float>());
    f.runsW64.assign(mixed ? 0 : nch, Run<double>());
    // S run: Sigma_SS with the training rows as right-hand sides
    const int Rn = (int)cdiv(n, TB);
    f.runS.add_problem(Ts, Rn, 0, false, -1);
    add_s_jtiles<double>(f.runS.rt, f.ptr<double>(f.o_Lss), f.ptr<double>(f.o_Ss64), s, d, Ts);
    for (int r = 0; r < Rn; ++r) {
      const int nv = (int)std::min<int64_t>(TB, n - (int64_t)r * TB);
      f.runS.rt.push_back(make_tile<double>(f.ptr<double>(f.o_Vt64) + (int64_t)r * TB * sp, sp, nullptr,
                                            f.ptr<double>(f.o_Xs64) + (int64_t)r * TB * d, nullptr, nv, nv,
                                            SRC_KERNEL, 0));
    }
    f.runS.schedule();
    // window runs (one per chunk) and the summary products
    auto window_runs = [&](auto& runs, auto& sums, auto* winbase, auto* cvec) {
      using TW = typename std::remove_const<typename std::remove_pointer<decltype(winbase)>::type>::type;
      for (int c = 0; c < nch; ++c) {
        build_window_run<TW>(f, runs[c], winbase, f.ptr<double>(f.o_Xs64), f.ptr<double>(f.o_Vt64), cvec,
                             f.ptr<double>(f.o_Ss64), use_band, f.chunk[c], f.chunk[c + 1]);
        runs[c].schedule();
      }
      f.sumsplit.assign(1, 0);
      if (nch == 1) {
        build_summary<TW>(f, sums, winbase);
      } else {
        f.sumout.clear();
        sums.clear();
        for (int c = 0; c < nch; ++c) {
          build_summary_chunk<TW>(f, sums, winbase, f.chunk[c], f.chunk[c + 1], c > 0);
          f.sumsplit.push_back((int64_t)f.sumout.size());
        }
        f.sumsplit.pop_back();
      }
      f.sumsplit.push_back((int64_t)f.sumout.size());
    };
    if (mixed)
      window_runs(f.runsW32, f.sum32, f.ptr<float>(f.o_win), f.ptr<float>(f.o_c32));
    else
      window_runs(f.runsW64, f.sum64, f.ptr<double>(f.o_win), f.ptr<double>(f.o_c64));
    // Sigma_ddot run (explicit matrix, no right-hand sides)
    f.runD.add_problem(Ts, 0, 0, false, -2);
    for (int i = 0; i < Ts; ++i) {
      const int nv = (int)std::min<int64_t>(TB, s - (int64_t)i * TB);
      RowTile<double> r = make_tile<double>(f.ptr<double>(f.o_Ldd) + jpanel_off(i), (int64_t)(i + 1) * TB, nullptr,
                                            nullptr, nullptr, nv, TB, SRC_EXPLICIT, 1);
      r.expl = f.ptr<double>(f.o_Sdd) + (int64_t)i * TB * sp;
      r.eld = sp;
      f.runD.rt.push_back(r);
    }
    f.runD.schedule();
    // kernel-times-vector items of the mixed refinement: c' = c - K_DS g over training
    // tiles, and r_X = c'_X - R_X beta_X over the tiles of every window
    f.kvcols.clear();
    f.kvcg.clear();
    f.kvkmv.clear();
    if (mixed) {
      const double* Xs = f.ptr<double>(f.o_Xs64);
      const double* Ss = f.ptr<double>(f.o_Ss64);
      kv_support_cols(f.kvcols, Ss, s, d, f.ptr<double>(f.o_g));
      const int ncs = (int)f.kvcols.size();
      for (int64_t r0 = 0; r0 < n; r0 += TB) {
        KvItem it = kv_item(Xs + r0 * d, (int)std::min<int64_t>(TB, n - r0), 0, ncs);
        it.base0 = f.ptr<double>(f.o_c64) + r0;
        it.out0 = f.ptr<double>(f.o_cg) + r0;
        f.kvcg.push_back(it);
      }
      int64_t vo = 0;
      f.kmvsplit.assign(M + 1, 0);
      for (int64_t m = 0; m < M; ++m) {
        f.kmvsplit[m] = (int64_t)f.kvkmv.size();
        const WinGeom g = win_geom(f.bp, M, f.B, m);
        const int c0 = (int)f.kvcols.size();
        kv_window_cols(f.kvcols, g, Xs, d, f.ptr<double>(f.o_xJ) + vo, f.ptr<double>(f.o_xW) + vo);
        const int c1 = (int)f.kvcols.size();
        for (int i = 0; i < g.T; ++i) {
          int nv;
          const int64_t pt = win_tile_point(g, i, &nv);
          KvItem it = kv_item(Xs + pt * d, nv, c0, c1);
          it.base0 = f.ptr<double>(f.o_cg) + pt;
          it.vt = f.ptr<double>(f.o_Vt64) + pt * sp;
          it.h0 = f.ptr<double>(f.o_hJ) + m * sp;
          it.h1 = f.ptr<double>(f.o_hW) + m * sp;
          it.self0 = f.ptr<double>(f.o_xJ) + vo + (int64_t)i * TB;
          it.self1 = f.ptr<double>(f.o_xW) + vo + (int64_t)i * TB;
          it.out0 = f.ptr<double>(f.o_tJ) + vo + (int64_t)i * TB;
          it.out1 = f.ptr<double>(f.o_tW) + vo + (int64_t)i * TB;
          it.flag = i < g.tw ? 1 : 0;
          f.kvkmv.push_back(it);
        }
        vo += (int64_t)g.T * TB;
      }
      f.kmvsplit[M] = (int64_t)f.kvkmv.size();
    }
  };
  auto runs_meta = [&]() {
    int64_t b = f.runS.meta_bytes() + f.runD.meta_bytes();
    for (auto& r : f.runsW32) b += r.meta_bytes();
    for (auto& r : f.runsW64) b += r.meta_bytes();
    return b;
  };
  int64_t meta = 0, sterm_bytes = 0;
  auto plan_meta = [&]() {
    build_runs(nullptr);
    meta = runs_meta();
    f.o_kvcols = ar.reserve(sizeof(KvCol) * std::max<size_t>(f.kvcols.size(), 1));
    f.o_kvcg = ar.reserve(sizeof(KvItem) * std::max<size_t>(f.kvcg.size(), 1));
    f.o_kvkmv = ar.reserve(sizeof(KvItem) * std::max<size_t>(f.kvkmv.size(), 1));
    sterm_bytes = mixed ? sizeof(GemmTerm<float>) * f.sum32.size() : sizeof(GemmTerm<double>) * f.sum64.size();
    f.o_meta = ar.reserve(meta);
    f.o_sumterms = ar.reserve(sterm_bytes);
    f.o_sumout = ar.reserve(sizeof(GemmOut) * f.sumout.size());
    f.ar.cap = f.ar.used;
  };
  plan_meta();
  const int64_t budget = p->mem_budget_bytes;
  if (budget > 0 && f.ar.cap > budget) {
    // Too small for every window's factors: keep one chunk of windows at a time.
    use_band = false;
    int64_t avail = budget - (f.ar.cap - wsz * (f.win_area + f.inv_area));
    bool ok = false;
    for (int attempt = 0; attempt < 4 && avail > 0; ++attempt) {
      if (!set_chunks(avail)) break;
      plan_fixed();
      plan_meta();
      if (f.ar.cap <= budget) {
        ok = true;
        break;
      }
      avail -= f.ar.cap - budget;
    }
    if (!ok) {
      char buf[200];
      snprintf(buf, sizeof buf, "mem_budget_bytes %lld is too small even for one window's factors at a time",
               (long long)budget);
      throw Err{LMA_E_NOMEM, buf};
    }
  }
  if (use_band && budget > 0 && f.ar.cap + bpl.bytes > budget) use_band = false;
  {
    void* mem = devcache::get((size_t)f.ar.cap);
    if (!mem) {
      char buf[160];
      snprintf(buf, sizeof buf, "hipMalloc of %lld bytes failed", (long long)f.ar.cap);
      throw Err{LMA_E_NOMEM, buf};
    }
    f.ar.used = f.ar.cap;
    if (use_band) {
      bpl.mem = devcache::get((size_t)bpl.bytes);
      bpl.st = st;
      if (!bpl.mem) use_band = false;  // not enough device memory: windows form their entries themselves
    }
    build_runs(reinterpret_cast<char*>(mem));
  }
  // ---- upload schedules
  {
    char* mp = f.ptr<char>(f.o_meta);
    f.runS.upload(mp, st);
    mp += f.runS.meta_bytes();
    for (auto& r : f.runsW32) {
      r.upload(mp, st);
      mp += r.meta_bytes();
    }
    for (auto& r : f.runsW64) {
      r.upload(mp, st);
      mp += r.meta_bytes();
    }
    f.runD.upload(mp, st);
    if (use_band) {
      char* bm = static_cast<char*>(bpl.mem);
      HIPCHK(hipMemcpyAsync(bm + bpl.o_items, bpl.items.data(), sizeof(BandItem) * bpl.items.size(),
                            hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(bm + bpl.o_brow, bpl.brow.data(), 8 * n, hipMemcpyHostToDevice, st));
    }
    if (mixed)
      HIPCHK(hipMemcpyAsync(f.ptr<char>(f.o_sumterms), f.sum32.data(), sterm_bytes, hipMemcpyHostToDevice, st));
    else
      HIPCHK(hipMemcpyAsync(f.ptr<char>(f.o_sumterms), f.sum64.data(), sterm_bytes, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(f.ptr<char>(f.o_sumout), f.sumout.data(), sizeof(GemmOut) * f.sumout.size(),
                          hipMemcpyHostToDevice, st));
    if (!f.kvcols.empty())
      HIPCHK(hipMemcpyAsync(f.ptr<char>(f.o_kvcols), f.kvcols.data(), sizeof(KvCol) * f.kvcols.size(),
                            hipMemcpyHostToDevice, st));
    if (!f.kvcg.empty())
      HIPCHK(hipMemcpyAsync(f.ptr<char>(f.o_kvcg), f.kvcg.data(), sizeof(KvItem) * f.kvcg.size(),
                            hipMemcpyHostToDevice, st));
    if (!f.kvkmv.empty())
      HIPCHK(hipMemcpyAsync(f.ptr<char>(f.o_kvkmv), f.kvkmv.data(), sizeof(KvItem) * f.kvkmv.size(),
                            hipMemcpyHostToDevice, st));
  }
  // ---- compute
  int32_t* status = f.ptr<int32_t>(f.o_status);
  double* logdiag = f.ptr<double>(f.o_logdiag);
  HIPCHK(hipMemsetAsync(status, 0, 4 * f.n_status, st));
  HIPCHK(hipMemsetAsync(logdiag, 0, 8 * f.n_logdiag, st));
  prof::timed(prof::OTHER, 0.0, st, [&] { launch_scale(p->X, n, (int)d, f.ie, f.ptr<double>(f.o_Xs64), nullptr, st); });
  prof::timed(prof::OTHER, 0.0, st, [&] { launch_scale(p->S, s, (int)d, f.ie, f.ptr<double>(f.o_Ss64), nullptr, st); });
  prof::timed(prof::OTHER, 0.0, st, [&] { launch_center(p->y, n, f.mu, f.ptr<double>(f.o_c64), f.ptr<float>(f.o_c32), st); });
  HIPCHK(hipGetLastError());
  const int maxTld = (int)(f.n_logdiag / (M + 2));
  // Runs share one logdiag stride (maxTld); set it before executing.
  auto run_with_stride = [&](auto& run, auto* invdiag, int slot, int vlen, bool with_band) {
    const int realT = run.maxT;
    using TT = typename std::remove_pointer<decltype(invdiag)>::type;
    StepArgs<TT> a{};
    if (with_band) {
      a.band = reinterpret_cast<const TT*>(bpl.mem);
      a.brow = reinterpret_cast<const int64_t*>(static_cast<char*>(bpl.mem) + bpl.o_brow);
    }
    a.rt = run.d_rt;
    a.pd = run.d_pd;
    a.vlen = vlen;
    a.vld = sp;
    a.d = (int)d;
    a.sf2 = f.sf2;
    a.sn2 = f.sn2;
    a.invdiag = invdiag;
    a.logdiag = logdiag + (int64_t)slot * maxTld;
    a.status = status + slot;
    a.maxT = maxTld;
    for (int j = 0; j < realT; ++j) {
      a.j = j;
      a.items = run.d_items + run.upd_off[j];
      a.nitems = (int32_t)run.upd_n[j];
      double f64 = 0.0;
      const double fl = prof::on ? run.update_flops(j, vlen > 0 ? s : 0, &f64) : 0.0;
      prof::timed(prof::UPDATE, fl, st, [&] { launch_update<TT>(a, std::is_same<TT, float>::value, st); }, f64);
      HIPCHK(hipGetLastError());
      prof::timed(prof::DIAG, 0.0, st, [&] { launch_diag<TT>(a, run.d_plist + run.pl_off[j], (int)run.pl_n[j], st); });
      HIPCHK(hipGetLastError());
      a.items = run.d_items + run.trs_off[j];
      a.nitems = (int32_t)run.trs_n[j];
      prof::timed(prof::TRSM, 0.0, st, [&] { launch_trsm<TT>(a, st); });
      HIPCHK(hipGetLastError());
    }
  };
  run_with_stride(f.runS, f.ptr<double>(f.o_Lss_inv), (int)M, 0, false);
  if (use_band) {
    auto band_launch = [&](auto* band) {
      using TT = typename std::remove_pointer<decltype(band)>::type;
      BandArgs<TT> ba{};
      ba.items = reinterpret_cast<const BandItem*>(static_cast<char*>(bpl.mem) + bpl.o_items);
      ba.nitems = (int32_t)bpl.items.size();
      ba.d = (int)d;
      ba.vlen = (int)sp;
      ba.vld = sp;
      ba.Vt = f.ptr<double>(f.o_Vt64);
      ba.Xs = f.ptr<double>(f.o_Xs64);
      ba.Vr = ba.Vt;
      ba.Xr = ba.Xs;
      ba.noise = 1;
      ba.sf2 = f.sf2;
      ba.sn2 = f.sn2;
      ba.band = band;
      double fl = 0.0;
      if (prof::on)
        for (const BandItem& it : bpl.items) fl += 2.0 * it.nr * it.nc * (double)s;
      prof::timed(prof::GEMM, fl, st, [&] { launch_band<TT>(ba, st); });
      HIPCHK(hipGetLastError());
    };
    if (mixed)
      band_launch(static_cast<float*>(bpl.mem));
    else
      band_launch(static_cast<double*>(bpl.mem));
  }
  const int nch = (int)f.chunk.size() - 1;
  // factor the windows of chunk c (their panels and inverses in the window area)
  auto factor_chunk = [&](int c) {
    if (mixed)
      run_with_stride(f.runsW32[c], f.ptr<float>(f.o_win_inv), (int)f.chunk[c], (int)sp, use_band);
    else
      run_with_stride(f.runsW64[c], f.ptr<double>(f.o_win_inv), (int)f.chunk[c], (int)sp, use_band);
  };
  for (int c = 0; c < nch; ++c) {
    factor_chunk(c);
    const int64_t o0 = f.sumsplit[c], o1 = f.sumsplit[c + 1];
    const GemmOut* douts = reinterpret_cast<const GemmOut*>(f.ptr<char>(f.o_sumout)) + o0;
    if (mixed)
      prof::timed(prof::GEMM, prof::on ? gemm_flops(f.sum32, f.sumout, o0, o1) : 0.0, st, [&] {
        launch_tile_gemm<float>(reinterpret_cast<const GemmTerm<float>*>(f.ptr<char>(f.o_sumterms)), douts,
                                (int)(o1 - o0), st);
      });
    else
      prof::timed(prof::GEMM, prof::on ? gemm_flops(f.sum64, f.sumout, o0, o1) : 0.0, st, [&] {
        launch_tile_gemm<double>(reinterpret_cast<const GemmTerm<double>*>(f.ptr<char>(f.o_sumterms)), douts,
                                 (int)(o1 - o0), st);
      });
    HIPCHK(hipGetLastError());
  }
  {
    SummaryArgs sa;
    sa.partial = f.ptr<double>(f.o_partial);
    sa.groups = f.groups;
    sa.ntile = f.ntile;
    sa.Ts = Ts;
    sa.sp = (int)sp;
    sa.s = (int)s;
    sa.d = (int)d;
    sa.Ss = f.ptr<double>(f.o_Ss64);
    sa.sf2 = f.sf2;
    sa.sn2 = f.sn2;
    sa.Sdd = f.ptr<double>(f.o_Sdd);
    sa.ydd = f.ptr<double>(f.o_ydd);
    sa.qsum = f.ptr<double>(f.o_q);
    prof::timed(prof::OTHER, 0.0, st, [&] { launch_finalize_summary(sa, st); });
    HIPCHK(hipGetLastError());
  }
  run_with_stride(f.runD, f.ptr<double>(f.o_Ldd_inv), (int)M + 1, 0, false);
  {
    SolveArgs so;
    so.L = f.ptr<double>(f.o_Ldd);
    so.inv = f.ptr<double>(f.o_Ldd_inv);
    so.A = f.ptr<double>(f.o_Sdd);
    so.b = f.ptr<double>(f.o_ydd);
    so.g = f.ptr<double>(f.o_g);
    so.sp = (int)sp;
    so.iters = 2;
    prof::timed(prof::OTHER, 0.0, st, [&] { launch_global_solve(so, st); });
    HIPCHK(hipGetLastError());
  }
  // ---- beta_X = R_X^-1 (c_X - K_XS g) for every window and separator
  {
    std::vector<int64_t> tab(10 * M);
    int64_t* t_wstart = tab.data();
    int64_t* t_wlen = t_wstart + M;
    int64_t* t_dstart = t_wlen + M;
    int64_t* t_dlen = t_dstart + M;
    int64_t* t_panel = t_dlen + M;
    int64_t* t_inv = t_panel + M;
    int64_t* t_vec = t_inv + M;
    int64_t* t_rhs = t_vec + M;
    int32_t* t_T = reinterpret_cast<int32_t*>(t_rhs + M);
    int32_t* t_tw = t_T + M;
    int64_t vec_acc = 0;
    int maxTw = 0;
    for (int64_t m = 0; m < M; ++m) {
      const WinGeom g = win_geom(f.bp, M, f.B, m);
      t_wstart[m] = g.wstart;
      t_wlen[m] = g.w;
      t_dstart[m] = g.dstart;
      t_dlen[m] = g.b;
      t_panel[m] = f.win_off[m];
      t_inv[m] = f.inv_off[m];
      t_vec[m] = vec_acc;
      t_rhs[m] = f.win_off[m] + jpanel_off(g.T);
      t_T[m] = g.T;
      t_tw[m] = g.tw;
      vec_acc += (int64_t)g.T * TB;
      maxTw = std::max(maxTw, g.T);
    }
    f.wt_host = tab;
    char* dt = f.ptr<char>(f.o_wt);
    HIPCHK(hipMemcpyAsync(dt, f.wt_host.data(), 8 * 10 * M, hipMemcpyHostToDevice, st));
    const int64_t* dtab = reinterpret_cast<const int64_t*>(dt);
    f.wt.wstart = dtab;
    f.wt.wlen = dtab + M;
    f.wt.dstart = dtab + 2 * M;
    f.wt.dlen = dtab + 3 * M;
    f.wt.panel = dtab + 4 * M;
    f.wt.inv = dtab + 5 * M;
    f.wt.vec = dtab + 6 * M;
    f.wt.rhs = dtab + 7 * M;
    f.wt.T = reinterpret_cast<const int32_t*>(dtab + 8 * M);
    f.wt.tw = f.wt.T + M;
    double* xJ = f.ptr<double>(f.o_xJ);
    double* xW = f.ptr<double>(f.o_xW);
    double* tJ = f.ptr<double>(f.o_tJ);
    double* tW = f.ptr<double>(f.o_tW);
    double* g = f.ptr<double>(f.o_g);
    HArgs ha;
    ha.w = f.wt;
    ha.Vt = f.ptr<double>(f.o_Vt64);
    ha.xJ = xJ;
    ha.xW = xW;
    ha.hJ = f.ptr<double>(f.o_hJ);
    ha.hW = f.ptr<double>(f.o_hW);
    ha.sp = (int)sp;
    ha.M = (int)M;
    // chunk c's windows m0..m1-1 seen by the kernels as windows 0..m1-m0-1
    auto sub = [&](int c) {
      const int64_t m0 = f.chunk[c];
      WinTab w = f.wt;
      w.wstart += m0;
      w.wlen += m0;
      w.dstart += m0;
      w.dlen += m0;
      w.panel += m0;
      w.inv += m0;
      w.vec += m0;
      w.rhs += m0;
      w.T += m0;
      w.tw += m0;
      return w;
    };
    auto nwin = [&](int c) { return (int)(f.chunk[c + 1] - f.chunk[c]); };
    auto h_chunk = [&](int c) {
      HArgs hc = ha;
      hc.w = sub(c);
      hc.M = nwin(c);
      hc.hJ = ha.hJ + f.chunk[c] * sp;
      hc.hW = ha.hW + f.chunk[c] * sp;
      prof::timed(prof::OTHER, 0.0, st, [&] { launch_h(hc, st); });
    };
    auto winvec = [&](auto* panels, auto* invs, double* vJ, double* vW, int c) {
      using TT = typename std::remove_const<typename std::remove_pointer<decltype(panels)>::type>::type;
      WinVecArgs<TT> va;
      va.w = sub(c);
      va.panels = panels;
      va.invs = invs;
      va.sp = (int)sp;
      va.s = (int)s;
      va.g = g;
      va.vJ = vJ;
      va.vW = vW;
      return va;
    };
    // beta from the whitened right-hand sides (forward half) and a backward solve
    auto beta_solve = [&](auto* panels, auto* invs, int c) {
      auto va = winvec(panels, invs, xJ, xW, c);
      using TT = typename std::remove_const<typename std::remove_pointer<decltype(panels)>::type>::type;
      prof::timed(prof::OTHER, 0.0, st, [&] { launch_ycp<TT>(va, nwin(c), maxTw, st); });
      prof::timed(prof::OTHER, 0.0, st, [&] { launch_bwd<TT>(va, nwin(c), st); });
      HIPCHK(hipGetLastError());
    };
    auto full_solve = [&](auto* panels, auto* invs, double* vJ, double* vW, int c) {
      auto va = winvec(panels, invs, vJ, vW, c);
      using TT = typename std::remove_const<typename std::remove_pointer<decltype(panels)>::type>::type;
      prof::timed(prof::OTHER, 0.0, st, [&] { launch_fwd<TT>(va, nwin(c), maxTw, st); });
      prof::timed(prof::OTHER, 0.0, st, [&] { launch_bwd<TT>(va, nwin(c), st); });
      HIPCHK(hipGetLastError());
    };
    // x += alpha t over the vector entries of chunk c's windows
    auto axpy_chunk = [&](double alpha, int c) {
      const int64_t v0 = t_vec[f.chunk[c]], v1 = f.chunk[c + 1] < M ? t_vec[f.chunk[c + 1]] : f.vec_elems;
      prof::timed(prof::OTHER, 0.0, st, [&] { launch_axpy2(xJ + v0, xW + v0, tJ + v0, tW + v0, alpha, v1 - v0, st); });
    };
    // the factors of chunk c are resident: with several chunks, factor them again
    auto resident = [&](int c) {
      if (nch > 1) factor_chunk(c);
    };
    if (!mixed) {
      for (int c = 0; c < nch; ++c) {
        resident(c);
        beta_solve(f.ptr<double>(f.o_win), f.ptr<double>(f.o_win_inv), c);
        h_chunk(c);
      }
      HIPCHK(hipGetLastError());
    } else {
      const float* P = f.ptr<float>(f.o_win);
      const float* I = f.ptr<float>(f.o_win_inv);
      double* cg = f.ptr<double>(f.o_cg);
      double* dg = f.ptr<double>(f.o_dg);
      double* tvec = f.ptr<double>(f.o_tvec);
      KvArgs kv;
      kv.cols = reinterpret_cast<const KvCol*>(f.ptr<char>(f.o_kvcols));
      kv.d = (int)d;
      kv.sp = (int)sp;
      kv.sf2 = f.sf2;
      kv.sn2 = f.sn2;
      kv.mu = 0.0;
      // c' = c - K_XS g over all training points
      kv.items = reinterpret_cast<const KvItem*>(f.ptr<char>(f.o_kvcg));
      kv.nitems = (int32_t)f.kvcg.size();
      kv.mode = KV_CG;
      prof::timed(prof::OTHER, 0.0, st, [&] { launch_kvec(kv, st); });
      for (int c = 0; c < nch; ++c) {
        resident(c);
        // 1. beta0 with the float32 factors
        beta_solve(P, I, c);
        h_chunk(c);
        // 2. one refinement of beta against the float64 residual covariance
        kv.items = reinterpret_cast<const KvItem*>(f.ptr<char>(f.o_kvkmv)) + f.kmvsplit[f.chunk[c]];
        kv.nitems = (int32_t)(f.kmvsplit[f.chunk[c + 1]] - f.kmvsplit[f.chunk[c]]);
        kv.mode = KV_KMV;
        prof::timed(prof::OTHER, 0.0, st, [&] { launch_kvec(kv, st); });
        full_solve(P, I, tJ, tW, c);
        axpy_chunk(1.0, c);
        h_chunk(c);
      }
      // 3. global correction: rho = y_ddot - Sigma_ddot g with exact window solves
      GresArgs gr;
      gr.L = f.ptr<double>(f.o_Lss);
      gr.hJ = ha.hJ;
      gr.hW = ha.hW;
      gr.g = g;
      gr.rho = f.ptr<double>(f.o_rho);
      gr.M = (int)M;
      gr.sp = (int)sp;
      prof::timed(prof::OTHER, 0.0, st, [&] { launch_gres(gr, st); });
      SolveArgs so;
      so.L = f.ptr<double>(f.o_Ldd);
      so.inv = f.ptr<double>(f.o_Ldd_inv);
      so.A = f.ptr<double>(f.o_Sdd);
      so.b = gr.rho;
      so.g = dg;
      so.sp = (int)sp;
      so.iters = 1;
      prof::timed(prof::OTHER, 0.0, st, [&] { launch_global_solve(so, st); });
      prof::timed(prof::OTHER, 0.0, st, [&] { launch_gupdate(gr.L, dg, g, tvec, (int)sp, st); });
      // 4. beta -= R_X^-1 K_XS dg  (K_XS dg = V_X^T L_SS^T dg); float32 factors suffice for the correction
      prof::timed(prof::OTHER, 0.0, st, [&] { launch_vdot(f.ptr<double>(f.o_Vt64), tvec, cg, n, (int)sp, st); });
      for (int c = 0; c < nch; ++c) {
        resident(c);
        const WinTab wc = sub(c);
        prof::timed(prof::OTHER, 0.0, st, [&] { launch_gather(wc, cg, tJ, tW, nwin(c), maxTw, st); });
        full_solve(P, I, tJ, tW, c);
        axpy_chunk(-1.0, c);
        h_chunk(c);
      }
      HIPCHK(hipGetLastError());
    }
  }
  // ---- read back status, log-diagonals, g, y_ddot, q
  std::vector<int32_t> hstat(f.n_status);
  std::vector<double> hld(f.n_logdiag);
  f.g.resize(sp);
  f.ydd.resize(sp);
  HIPCHK(hipMemcpyAsync(hstat.data(), status, 4 * f.n_status, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hld.data(), logdiag, 8 * f.n_logdiag, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(f.g.data(), f.ptr<double>(f.o_g), 8 * sp, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(f.ydd.data(), f.ptr<double>(f.o_ydd), 8 * sp, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&f.qsum, f.ptr<double>(f.o_q), 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  prof::flush();
  if (const char* dump = std::getenv("LMA_DUMP_WINDOW")) {  // diagnostic: "m:path" writes window m's panel
    const int64_t m = std::atoll(dump);
    const char* path = std::strchr(dump, ':');
    if (path && m >= 0 && m < M) {
      const int64_t el = panel_elems(f.Tm[m], Ts + 1);
      std::vector<char> h((size_t)(el * wsz));
      HIPCHK(hipMemcpy(h.data(), f.ptr<char>(f.o_win) + f.win_off[m] * wsz, h.size(), hipMemcpyDeviceToHost));
      if (FILE* fp = std::fopen(path + 1, "wb")) {
        const int64_t hdr[4] = {f.Tm[m], f.twm[m], Ts, wsz};
        std::fwrite(hdr, sizeof hdr, 1, fp);
        std::fwrite(h.data(), 1, h.size(), fp);
        std::fclose(fp);
      }
    }
  }
  if (hstat[M]) {
    g_failed = -1;
    throw Err{LMA_E_NOT_PD, "Sigma_SS is not positive definite"};
  }
  for (int64_t m = 0; m < M; ++m)
    if (hstat[m]) {
      g_failed = m;
      char buf[128];
      snprintf(buf, sizeof buf, "residual covariance of the window of block %lld is not positive definite",
               (long long)m);
      throw Err{LMA_E_NOT_PD, buf};
    }
  if (hstat[M + 1]) {
    g_failed = -2;
    throw Err{LMA_E_NOT_PD, "Sigma_ddot_SS is not positive definite"};
  }
  // log-determinants (fixed summation order)
  double ldR = 0;
  for (int64_t m = 0; m < M; ++m)
    for (int j = 0; j < f.Tm[m]; ++j) ldR += hld[(int64_t)m * maxTld + j];
  double lss = 0, ldd = 0;
  for (int j = 0; j < Ts; ++j) {
    lss += hld[(int64_t)M * maxTld + j];
    ldd += hld[(int64_t)(M + 1) * maxTld + j];
  }
  f.ld_R = 2 * ldR;
  f.ld_ss = 2 * lss;
  f.ld_dd = 2 * ldd;
  double ydg = 0;
  for (int64_t i = 0; i < sp; ++i) ydg += f.ydd[i] * f.g[i];
  f.ydg = ydg;
  f.lml = -0.5 * (f.qsum - ydg + f.ld_R + f.ld_dd - f.ld_ss + (double)n * std::log(2.0 * M_PI));
  if (!std::isfinite(f.lml)) throw Err{LMA_E_NOT_PD, "non-finite log marginal likelihood"};
  (void)keep;
  *out = F.release();
  return LMA_OK;
}

// ---------------------------------------------------------------------------
// predict
// ---------------------------------------------------------------------------
template <typename TW>
void predict_windows(lma_state& f, Run<TW>& run, int64_t n_u, const std::vector<int64_t>& ubp, const double* Us,
                     const double* VtU, TW* Xbuf, const std::vector<int64_t>& Xoff, TW* winbase, const double* Xs,
                     const double* Vt, const TW* c, int64_t m0, int64_t m1, bool refactor, bool tband) {
  const int Ts = (int)f.Ts;
  for (int64_t m = m0; m < m1; ++m) {
    const WinGeom g = win_geom(f.bp, f.M, f.B, m);
    const int64_t qhi = std::min(m + f.B, f.M - 1);
    const int64_t r0 = ubp[m], nr = ubp[qhi + 1] - ubp[m];
    if (nr <= 0) continue;
    const int R = (int)cdiv(nr, TB);
    const int64_t ld = (int64_t)g.T * TB;
    run.add_problem(g.T, R + (refactor ? Ts + 1 : 0), g.tw, !refactor, (int)m);
    // the window's rows: the stored factor (solve-only), or generated again with
    // its support rows and output row so that the factor and the whitened
    // right-hand sides are rebuilt as in the fit
    add_window_jtiles<TW>(run.rt, g, winbase + f.win_off[m], Xs, Vt, c, f.d, f.sp);
    run.pd.back().invdiag_off = win_inv_off(f, m);
    if (refactor) {
      TW* rhs = winbase + f.win_off[m] + jpanel_off(g.T);
      for (int r = 0; r < Ts; ++r) {
        const int nv = (int)std::min<int64_t>(TB, f.s - (int64_t)r * TB);
        const bool f64 = std::is_same<TW, double>::value;
        const double* Ss = f.ptr<double>(f.o_Ss64);
        RowTile<TW> t = make_tile<TW>(rhs + (int64_t)r * TB * ld, ld, nullptr,
                                      f64 ? reinterpret_cast<const TW*>(Ss + (int64_t)r * TB * f.d) : nullptr,
                                      nullptr, nv, TB, SRC_KERNEL, 0);
        t.xs64 = Ss + (int64_t)r * TB * f.d;
        run.rt.push_back(t);
      }
      run.rt.push_back(make_tile<TW>(rhs + (int64_t)Ts * TB * ld, ld, nullptr, nullptr, nullptr, 1, TB, SRC_CVEC, 0));
    }
    for (int r = 0; r < R; ++r) {
      const int nv = (int)std::min<int64_t>(TB, nr - (int64_t)r * TB);
      const int64_t pt = r0 + (int64_t)r * TB;
      const bool f64 = std::is_same<TW, double>::value;
      RowTile<TW> t = make_tile<TW>(Xbuf + Xoff[m] + (int64_t)r * TB * ld, ld,
                                    f64 ? reinterpret_cast<const TW*>(VtU + pt * f.sp) : nullptr,
                                    f64 ? reinterpret_cast<const TW*>(Us + pt * f.d) : nullptr, nullptr, nv, nv,
                                    SRC_KERNEL, 0);
      t.vt64 = VtU + pt * f.sp;
      t.xs64 = Us + pt * f.d;
      t.pt0 = pt;
      if (tband) t.src = SRC_TBAND;
      run.rt.push_back(t);
    }
  }
  (void)n_u;
}

}  // namespace


template <typename TW>
static void predict_impl(lma_state& f, int64_t n_u, const double* U, const int64_t* u_block_ptr, double* mean,
                         double* var, hipStream_t st, double* cov = nullptr) {
  const int64_t d = f.d, sp = f.sp, M = f.M;
  const int Ts = (int)f.Ts;
  const bool mixed = f.mixed();
  std::vector<int64_t> ubp(u_block_ptr, u_block_ptr + M + 1);
  // The full covariance needs everything the variance needs (whitened test
  // rows of every window, L_ddot^-1 E_u); without caller buffers for the mean
  // or the variance they live in the workspace.
  const bool want_cov = cov != nullptr;
  const bool need_var = var != nullptr || want_cov;
  // With the window factors held one chunk at a time (memory budget), each
  // chunk is factored again with the test rows appended, and the test rows'
  // solutions are kept for one chunk at a time.
  const bool stream = f.streaming();
  const int nch = stream ? (int)f.chunk.size() - 1 : 1;
  // Test band: R_ux for every test point u of block q and every training point x
  // of blocks q-B .. q+B (all windows that hold u lie there), formed once and
  // read by the B+1 window solves of u (not in the memory-budget mode).
  const int64_t wsz = (int64_t)sizeof(TW);
  const bool use_tband = need_var && n_u > 0 && !stream && std::getenv("LMA_NO_BAND") == nullptr;
  std::vector<BandItem> tb_items;
  std::vector<int64_t> tb_row;
  int64_t tb_elems = 0;
  if (use_tband) {
    tb_row.resize(n_u);
    for (int64_t q = 0; q < M; ++q) {
      const int64_t r0 = ubp[q], r1 = ubp[q + 1];
      if (r1 <= r0) continue;
      const int64_t c0 = f.bp[std::max<int64_t>(0, q - f.B)], c1 = f.bp[std::min<int64_t>(M - 1, q + f.B) + 1];
      const int64_t w = c1 - c0;
      for (int64_t u = r0; u < r1; ++u) tb_row[u] = tb_elems + (u - r0) * w - c0;
      for (int64_t g0 = r0; g0 < r1; g0 += 4 * TB) {
        const int64_t g1 = std::min<int64_t>(r1, g0 + 4 * TB);
        for (int64_t x0 = c0; x0 < c1; x0 += TB)
          for (int64_t u0 = g0; u0 < g1; u0 += TB) {
            BandItem it;
            it.p0 = u0;
            it.q0 = x0;
            it.off = tb_elems + (u0 - r0) * w + (x0 - c0);
            it.ld = w;
            it.nr = (int)std::min<int64_t>(TB, r1 - u0);
            it.nc = (int)std::min<int64_t>(TB, c1 - x0);
            tb_items.push_back(it);
          }
      }
      tb_elems += (r1 - r0) * w;
    }
  }
  std::vector<int64_t> pchunk = stream ? f.chunk : std::vector<int64_t>{0, M};
  // window geometry for test rows
  std::vector<int64_t> Xoff(M, 0);
  int64_t xel = 0;
  for (int ci = 0; ci < nch; ++ci) {
    int64_t acc = 0;
    for (int64_t m = pchunk[ci]; m < pchunk[ci + 1]; ++m) {
      const int64_t qhi = std::min(m + f.B, M - 1);
      const int64_t nr = ubp[qhi + 1] - ubp[m];
      Xoff[m] = acc;
      if (need_var) acc += nr * (int64_t)f.Tm[m] * TB;
    }
    xel = std::max(xel, acc);
  }
  int maxT = 1;
  for (int64_t m = 0; m < M; ++m) maxT = std::max(maxT, (int)f.Tm[m]);
  const int64_t ldG = sp + TB;
  Arena ar;
  const int64_t o_Us64 = ar.reserve(8 * n_u * d);
  const int64_t o_VtU64 = ar.reserve(8 * n_u * sp);
  const int64_t o_X = ar.reserve((int64_t)sizeof(TW) * xel);
  const int64_t o_G = ar.reserve(8 * n_u * ldG);
  const int64_t o_vn = ar.reserve(8 * n_u);
  const int64_t o_xi = ar.reserve(8 * n_u);
  const int64_t o_ublk = ar.reserve(4 * n_u);
  const int64_t o_uptr = ar.reserve(8 * (M + 1));
  const int64_t o_Xoff = ar.reserve(8 * M);
  const int64_t o_Tm = ar.reserve(4 * M);
  const int64_t o_twm = ar.reserve(4 * M);
  const int64_t o_stat = ar.reserve(4 * (M + 2));
  const int64_t o_ld = ar.reserve(8 * (M + 2) * (int64_t)maxT);  // log-diagonals of refactored windows
  const int64_t o_mtmp = mean ? 0 : ar.reserve(8 * n_u);
  const int64_t o_vtmp = (want_cov && !var) ? ar.reserve(8 * n_u) : 0;
  double* mean_p = mean;
  double* var_p = var;
  // full covariance: residual entries of the test pairs inside the band
  // (k_band with the test points as rows and columns), the low-rank term
  // (L_ddot^-1 E)^T (L_ddot^-1 E) over every tile pair, and the whitened
  // products xi of the windows that hold both points of a pair
  std::vector<BandItem> cb_items;
  std::vector<GemmTerm<double>> cterms;
  std::vector<GemmOut> couts;
  std::vector<GemmTerm<TW>> xterms;
  std::vector<GemmOut> xouts;
  std::vector<int> xsplit;   // xi outputs of chunk ci: [xsplit[ci], xsplit[ci+1])
  if (want_cov) {
    for (int64_t q = 0; q < M; ++q)
      for (int64_t r = std::max<int64_t>(0, q - f.B); r <= std::min<int64_t>(M - 1, q + f.B); ++r)
        for (int64_t u0 = ubp[q]; u0 < ubp[q + 1]; u0 += TB)
          for (int64_t v0 = ubp[r]; v0 < ubp[r + 1]; v0 += TB) {
            BandItem it;
            it.p0 = u0;
            it.q0 = v0;
            it.off = u0 * n_u + v0;
            it.ld = n_u;
            it.nr = (int)std::min<int64_t>(TB, ubp[q + 1] - u0);
            it.nc = (int)std::min<int64_t>(TB, ubp[r + 1] - v0);
            cb_items.push_back(it);
          }
  }
  // runs
  Run<double> runS;
  std::vector<Run<TW>> runsW(nch);
  Run<double> runD;
  std::vector<GemmTerm<TW>> terms;
  std::vector<GemmOut> outs;
  std::vector<int> gsplit;  // streaming: G outputs of chunk ci, delta dl: [gsplit[k], gsplit[k+1]), k = ci*(B+1)+dl
  std::vector<KvCol> kvcols;
  std::vector<KvItem> kvitems;
  const int64_t o_hq = ar.reserve(8 * M * sp);
  const int64_t o_tb = ar.reserve(wsz * std::max<int64_t>(tb_elems, 1));
  const int64_t o_tbi = ar.reserve((int64_t)sizeof(BandItem) * std::max<int64_t>((int64_t)tb_items.size(), 1));
  const int64_t o_tbr = ar.reserve(8 * std::max<int64_t>((int64_t)tb_row.size(), 1));
  auto build = [&](char* base) {
    ar.base = base;
    runS = Run<double>();
    runsW.assign(nch, Run<TW>());
    runD = Run<double>();
    terms.clear();
    outs.clear();
    kvcols.clear();
    kvitems.clear();
    cterms.clear();
    couts.clear();
    xterms.clear();
    xouts.clear();
    xsplit.clear();
    if (!mean) mean_p = at<double>(ar, o_mtmp);
    if (want_cov && !var) var_p = at<double>(ar, o_vtmp);
    // S run in solve-only mode: right-hand sides are the test rows -> V_U^T
    const int Rn = (int)cdiv(n_u, TB);
    runS.add_problem(Ts, Rn, 0, true, -1);
    add_s_jtiles<double>(runS.rt, f.ptr<double>(f.o_Lss), f.ptr<double>(f.o_Ss64), f.s, d, Ts);
    for (int r = 0; r < Rn; ++r) {
      const int nv = (int)std::min<int64_t>(TB, n_u - (int64_t)r * TB);
      runS.rt.push_back(make_tile<double>(at<double>(ar, o_VtU64) + (int64_t)r * TB * sp, sp, nullptr,
                                          at<double>(ar, o_Us64) + (int64_t)r * TB * d, nullptr, nv, nv, SRC_KERNEL,
                                          0));
    }
    runS.schedule();
    // predictive mean: per test tile of block q, the support tiles with g, the J_m tiles
    // of windows m = q-B..q with beta_J and (m < q) the W_m tiles with beta_W
    {
      const double* Xs64 = f.ptr<double>(f.o_Xs64);
      for (int64_t q = 0; q < M; ++q) {
        if (ubp[q + 1] == ubp[q]) continue;
        const int c0 = (int)kvcols.size();
        kv_support_cols(kvcols, f.ptr<double>(f.o_Ss64), f.s, d, f.ptr<double>(f.o_g));
        for (int64_t dl = 0; dl <= f.B && dl <= q; ++dl) {
          const int64_t m = q - dl;
          const int64_t vo = f.wt_host[6 * M + m];
          kv_window_cols(kvcols, win_geom(f.bp, M, f.B, m), Xs64, d, f.ptr<double>(f.o_xJ) + vo,
                         dl > 0 ? f.ptr<double>(f.o_xW) + vo : nullptr);
        }
        const int c1 = (int)kvcols.size();
        for (int64_t u0 = ubp[q]; u0 < ubp[q + 1]; u0 += TB) {
          KvItem it = kv_item(at<double>(ar, o_Us64) + u0 * d, (int)std::min<int64_t>(TB, ubp[q + 1] - u0), c0, c1);
          it.vt = at<double>(ar, o_VtU64) + u0 * sp;
          it.h0 = at<double>(ar, o_hq) + q * sp;
          it.out0 = mean_p + u0;
          kvitems.push_back(it);
        }
      }
    }
    // window runs in solve-only mode
    const double* Us = at<double>(ar, o_Us64);
    const double* VtU = at<double>(ar, o_VtU64);
    const double* Xs = f.ptr<double>(f.o_Xs64);
    const double* Vt = f.ptr<double>(f.o_Vt64);
    const TW* c = mixed ? (const TW*)f.ptr<float>(f.o_c32) : (const TW*)f.ptr<double>(f.o_c64);
    TW* winbase = reinterpret_cast<TW*>(f.ptr<char>(f.o_win));
    if (!var_p) return;
    for (int ci = 0; ci < nch; ++ci) {
      predict_windows<TW>(f, runsW[ci], n_u, ubp, Us, VtU, at<TW>(ar, o_X), Xoff, winbase, Xs, Vt, c, pchunk[ci],
                          pchunk[ci + 1], stream, use_tband);
      runsW[ci].schedule();
    }
    // G accumulation: window m contributes to test blocks q = m..m+B (delta = q - m)
    auto g_term = [&](int64_t m, int64_t q, bool accumulate) {
      const int64_t dl = q - m;
      const int64_t uq = ubp[q + 1] - ubp[q];
      if (uq <= 0) return;
      const WinGeom g = win_geom(f.bp, M, f.B, m);
      const int64_t ldx = (int64_t)g.T * TB;
      const TW* Xm = at<TW>(ar, o_X) + Xoff[m] + (ubp[q] - ubp[m]) * ldx;
      const TW* rhs = winbase + f.win_off[m] + jpanel_off(g.T);
      for (int64_t t = 0; t < cdiv(uq, TB); ++t) {
        const int rows = (int)std::min<int64_t>(TB, uq - t * TB);
        for (int b = 0; b <= Ts; ++b) {
          GemmOut o = gemm_out(at<double>(ar, o_G) + (ubp[q] + t * TB) * ldG + (int64_t)b * TB, ldG, rows, TB,
                               accumulate ? 1 : 0, (int)terms.size());
          GemmTerm<TW> tm;
          tm.a = Xm + t * TB * ldx;
          tm.lda = ldx;
          tm.anr = rows;
          tm.b = rhs + (int64_t)b * TB * ldx;
          tm.ldb = ldx;
          tm.bnr = TB;
          tm.k0 = dl == 0 ? 0 : g.tw * TB;
          tm.k1 = g.T * TB;
          terms.push_back(tm);
          o.t1 = (int32_t)terms.size();
          outs.push_back(o);
        }
      }
    };
    if (!stream) {
      // by delta, so that delta = 0 writes each test row's G first
      for (int dl = 0; dl <= f.B; ++dl)
        for (int64_t q = dl; q < M; ++q) g_term(q - dl, q, dl > 0);
    } else {
      // by chunk of windows, then by delta (G cleared beforehand): within one
      // launch every window writes different test rows
      gsplit.assign(1, 0);
      for (int ci = 0; ci < nch; ++ci)
        for (int dl = 0; dl <= f.B; ++dl) {
          for (int64_t m = pchunk[ci]; m < pchunk[ci + 1] && m + dl < M; ++m) g_term(m, m + dl, true);
          gsplit.push_back((int)outs.size());
        }
    }
    // Sigma_ddot run in solve-only mode: right-hand sides E_u = k_u - G_u (in place)
    const int Ru = (int)cdiv(n_u, TB);
    runD.add_problem(Ts, Ru, 0, true, -2);
    for (int i = 0; i < Ts; ++i) {
      const int nv = (int)std::min<int64_t>(TB, f.s - (int64_t)i * TB);
      RowTile<double> r = make_tile<double>(f.ptr<double>(f.o_Ldd) + jpanel_off(i), (int64_t)(i + 1) * TB, nullptr,
                                            nullptr, nullptr, nv, TB, SRC_EXPLICIT, 1);
      r.expl = f.ptr<double>(f.o_Sdd) + (int64_t)i * TB * sp;
      r.eld = sp;
      runD.rt.push_back(r);
    }
    for (int r = 0; r < Ru; ++r) {
      const int nv = (int)std::min<int64_t>(TB, n_u - (int64_t)r * TB);
      double* rows = at<double>(ar, o_G) + (int64_t)r * TB * ldG;
      RowTile<double> t = make_tile<double>(rows, ldG, nullptr, nullptr, nullptr, nv, nv, SRC_EXPLICIT, 0);
      t.expl = rows;
      t.eld = ldG;
      runD.rt.push_back(t);
    }
    runD.schedule();
    if (!want_cov) return;
    // low-rank term over every tile pair: rows of L_ddot^-1 E (the Sigma_ddot
    // run's right-hand sides, in place in G)
    for (int64_t u0 = 0; u0 < n_u; u0 += TB)
      for (int64_t v0 = 0; v0 < n_u; v0 += TB) {
        const int rows = (int)std::min<int64_t>(TB, n_u - u0), cols = (int)std::min<int64_t>(TB, n_u - v0);
        GemmOut o = gemm_out(cov + u0 * n_u + v0, n_u, rows, cols, 1, (int)cterms.size());
        GemmTerm<double> tm;
        tm.a = at<double>(ar, o_G) + u0 * ldG;
        tm.lda = ldG;
        tm.anr = rows;
        tm.b = at<double>(ar, o_G) + v0 * ldG;
        tm.ldb = ldG;
        tm.bnr = cols;
        tm.k0 = 0;
        tm.k1 = (int32_t)sp;
        cterms.push_back(tm);
        o.t1 = (int32_t)cterms.size();
        couts.push_back(o);
      }
    // xi of the pair tiles (u in block q, v in block r, |q - r| <= B; a = min,
    // b = max): D rows of windows max(0, b-B) .. a-1, all rows of window a;
    // subtracted.  One output per tile pair and chunk of windows.
    xsplit.assign(1, 0);
    for (int ci = 0; ci < nch; ++ci) {
      for (int64_t q = 0; q < M; ++q)
        for (int64_t r = std::max<int64_t>(0, q - f.B); r <= std::min<int64_t>(M - 1, q + f.B); ++r) {
          const int64_t a = std::min(q, r), b = std::max(q, r);
          const int64_t m0 = std::max<int64_t>({(int64_t)0, b - f.B, pchunk[ci]});
          const int64_t m1 = std::min<int64_t>(a + 1, pchunk[ci + 1]);
          if (m0 >= m1) continue;
          for (int64_t u0 = ubp[q]; u0 < ubp[q + 1]; u0 += TB)
            for (int64_t v0 = ubp[r]; v0 < ubp[r + 1]; v0 += TB) {
              const int rows = (int)std::min<int64_t>(TB, ubp[q + 1] - u0);
              const int cols = (int)std::min<int64_t>(TB, ubp[r + 1] - v0);
              GemmOut o = gemm_out(cov + u0 * n_u + v0, n_u, rows, cols, 1, (int)xterms.size());
              for (int64_t m = m0; m < m1; ++m) {
                const WinGeom g = win_geom(f.bp, M, f.B, m);
                const int64_t ldx = (int64_t)g.T * TB;
                const TW* Xm = at<TW>(ar, o_X) + Xoff[m];
                GemmTerm<TW> tm;
                tm.a = Xm + (u0 - ubp[m]) * ldx;
                tm.lda = ldx;
                tm.anr = rows;
                tm.b = Xm + (v0 - ubp[m]) * ldx;
                tm.ldb = ldx;
                tm.bnr = cols;
                tm.k0 = m == a ? 0 : g.tw * TB;
                tm.k1 = g.T * TB;
                xterms.push_back(tm);
              }
              o.tneg = o.t1 = (int32_t)xterms.size();
              xouts.push_back(o);
            }
        }
      xsplit.push_back((int)xouts.size());
    }
  };
  build(nullptr);
  // dG outputs: one launch per delta; record split points
  std::vector<int> dl_split(f.B + 2, 0);
  {
    int idx = 0;
    for (int dl = 0; dl <= f.B; ++dl) {
      dl_split[dl] = idx;
      for (int64_t q = dl; q < M; ++q) {
        const int64_t uq = ubp[q + 1] - ubp[q];
        if (uq <= 0) continue;
        idx += (int)cdiv(uq, TB) * (Ts + 1);
      }
    }
    dl_split[f.B + 1] = idx;
  }
  int64_t wmeta = 0;
  for (auto& r : runsW) wmeta += r.meta_bytes();
  const int64_t o_meta = ar.reserve(runS.meta_bytes() + wmeta + runD.meta_bytes());
  const int64_t o_kvc = ar.reserve(sizeof(KvCol) * std::max<size_t>(kvcols.size(), 1));
  const int64_t o_kvi = ar.reserve(sizeof(KvItem) * std::max<size_t>(kvitems.size(), 1));
  const int64_t o_terms = ar.reserve(sizeof(GemmTerm<TW>) * std::max<size_t>(terms.size(), 1));
  const int64_t o_outs = ar.reserve(sizeof(GemmOut) * std::max<size_t>(outs.size(), 1));
  const int64_t o_cbi = ar.reserve(sizeof(BandItem) * std::max<size_t>(cb_items.size(), 1));
  const int64_t o_cterms = ar.reserve(sizeof(GemmTerm<double>) * std::max<size_t>(cterms.size(), 1));
  const int64_t o_couts = ar.reserve(sizeof(GemmOut) * std::max<size_t>(couts.size(), 1));
  const int64_t o_xterms = ar.reserve(sizeof(GemmTerm<TW>) * std::max<size_t>(xterms.size(), 1));
  const int64_t o_xouts = ar.reserve(sizeof(GemmOut) * std::max<size_t>(xouts.size(), 1));
  ar.cap = ar.used;
  void* mem = devcache::get((size_t)ar.cap);
  if (!mem) throw Err{LMA_E_NOMEM, "device allocation of the prediction workspace failed"};
  struct Guard {
    void* p;
    size_t bytes;
    hipStream_t s;
    ~Guard() {
      if (p) {
        (void)hipStreamSynchronize(s);
        devcache::put(p, bytes);
      }
    }
  } guard{mem, (size_t)ar.cap, st};
  build(reinterpret_cast<char*>(mem));
  {
    char* mp = at<char>(ar, o_meta);
    runS.upload(mp, st);
    mp += runS.meta_bytes();
    for (auto& r : runsW) {
      r.upload(mp, st);
      mp += r.meta_bytes();
    }
    runD.upload(mp, st);
    if (!terms.empty())
      HIPCHK(hipMemcpyAsync(at<char>(ar, o_terms), terms.data(), sizeof(GemmTerm<TW>) * terms.size(),
                            hipMemcpyHostToDevice, st));
    if (!outs.empty())
      HIPCHK(hipMemcpyAsync(at<char>(ar, o_outs), outs.data(), sizeof(GemmOut) * outs.size(), hipMemcpyHostToDevice,
                            st));
    if (!kvcols.empty())
      HIPCHK(hipMemcpyAsync(at<char>(ar, o_kvc), kvcols.data(), sizeof(KvCol) * kvcols.size(), hipMemcpyHostToDevice,
                            st));
    if (!kvitems.empty())
      HIPCHK(hipMemcpyAsync(at<char>(ar, o_kvi), kvitems.data(), sizeof(KvItem) * kvitems.size(),
                            hipMemcpyHostToDevice, st));
    if (!cb_items.empty())
      HIPCHK(hipMemcpyAsync(at<char>(ar, o_cbi), cb_items.data(), sizeof(BandItem) * cb_items.size(),
                            hipMemcpyHostToDevice, st));
    if (!cterms.empty()) {
      HIPCHK(hipMemcpyAsync(at<char>(ar, o_cterms), cterms.data(), sizeof(GemmTerm<double>) * cterms.size(),
                            hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(at<char>(ar, o_couts), couts.data(), sizeof(GemmOut) * couts.size(),
                            hipMemcpyHostToDevice, st));
    }
    if (!xterms.empty()) {
      HIPCHK(hipMemcpyAsync(at<char>(ar, o_xterms), xterms.data(), sizeof(GemmTerm<TW>) * xterms.size(),
                            hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(at<char>(ar, o_xouts), xouts.data(), sizeof(GemmOut) * xouts.size(),
                            hipMemcpyHostToDevice, st));
    }
  }
  std::vector<int32_t> ublk(n_u);
  for (int64_t q = 0; q < M; ++q)
    for (int64_t u = ubp[q]; u < ubp[q + 1]; ++u) ublk[u] = (int32_t)q;
  std::vector<int64_t> Xoff_h(Xoff);
  HIPCHK(hipMemcpyAsync(at<char>(ar, o_ublk), ublk.data(), 4 * n_u, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(at<char>(ar, o_uptr), ubp.data(), 8 * (M + 1), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(at<char>(ar, o_Xoff), Xoff_h.data(), 8 * M, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(at<char>(ar, o_Tm), f.Tm.data(), 4 * M, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(at<char>(ar, o_twm), f.twm.data(), 4 * M, hipMemcpyHostToDevice, st));
  if (use_tband) {
    HIPCHK(hipMemcpyAsync(at<char>(ar, o_tbi), tb_items.data(), sizeof(BandItem) * tb_items.size(),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(at<char>(ar, o_tbr), tb_row.data(), 8 * tb_row.size(), hipMemcpyHostToDevice, st));
  }
  int32_t* stat = at<int32_t>(ar, o_stat);
  double* ldg = at<double>(ar, o_ld);
  HIPCHK(hipMemsetAsync(stat, 0, 4 * (M + 2), st));
  // scale test inputs
  prof::timed(prof::OTHER, 0.0, st, [&] { launch_scale(U, n_u, (int)d, f.ie, at<double>(ar, o_Us64), nullptr, st); });
  HIPCHK(hipGetLastError());
  auto exec = [&](auto& run, auto* invdiag, int vlen, bool factor = false, bool with_tband = false) {
    using TT = typename std::remove_pointer<decltype(invdiag)>::type;
    StepArgs<TT> a{};
    if (with_tband) {
      a.band = at<TT>(ar, o_tb);
      a.brow = at<int64_t>(ar, o_tbr);
    }
    a.rt = run.d_rt;
    a.pd = run.d_pd;
    a.vlen = vlen;
    a.vld = sp;
    a.d = (int)d;
    a.sf2 = f.sf2;
    a.sn2 = f.sn2;
    a.invdiag = invdiag;
    a.logdiag = ldg;
    a.status = stat;
    a.maxT = maxT;
    for (int j = 0; j < run.maxT; ++j) {
      a.j = j;
      a.items = run.d_items + run.upd_off[j];
      a.nitems = (int32_t)run.upd_n[j];
      double f64 = 0.0;
      const double fl = prof::on ? run.update_flops(j, vlen > 0 ? f.s : 0, &f64) : 0.0;
      prof::timed(prof::UPDATE, fl, st, [&] { launch_update<TT>(a, std::is_same<TT, float>::value, st); }, f64);
      HIPCHK(hipGetLastError());
      if (factor) {
        prof::timed(prof::DIAG, 0.0, st, [&] { launch_diag<TT>(a, run.d_plist + run.pl_off[j], (int)run.pl_n[j], st); });
        HIPCHK(hipGetLastError());
      }
      a.items = run.d_items + run.trs_off[j];
      a.nitems = (int32_t)run.trs_n[j];
      prof::timed(prof::TRSM, 0.0, st, [&] { launch_trsm<TT>(a, st); });
      HIPCHK(hipGetLastError());
    }
  };
  exec(runS, f.ptr<double>(f.o_Lss_inv), 0);
  {
    prof::timed(prof::OTHER, 0.0, st, [&] {
      launch_hq(f.ptr<double>(f.o_hJ), f.ptr<double>(f.o_hW), at<double>(ar, o_hq), (int)M, (int)f.B, (int)sp, st);
    });
    KvArgs kv;
    kv.items = at<KvItem>(ar, o_kvi);
    kv.cols = at<KvCol>(ar, o_kvc);
    kv.nitems = (int32_t)kvitems.size();
    kv.mode = KV_MEAN;
    kv.d = (int)d;
    kv.sp = (int)sp;
    kv.sf2 = f.sf2;
    kv.sn2 = f.sn2;
    kv.mu = f.mu;
    prof::timed(prof::OTHER, 0.0, st, [&] { launch_kvec(kv, st); });
    HIPCHK(hipGetLastError());
  }
  if (want_cov) {
    // covariance: zero, then the residual entries of the in-band pairs
    prof::timed(prof::OTHER, 0.0, st, [&] { launch_zero(cov, n_u * n_u, st); });
    HIPCHK(hipGetLastError());
    BandArgs<double> cb{};
    cb.items = at<BandItem>(ar, o_cbi);
    cb.nitems = (int32_t)cb_items.size();
    cb.d = (int)d;
    cb.vlen = (int)sp;
    cb.noise = 1;  // one point set: sn2 on the diagonal
    cb.vld = sp;
    cb.Vt = at<double>(ar, o_VtU64);
    cb.Xs = at<double>(ar, o_Us64);
    cb.Vr = at<double>(ar, o_VtU64);
    cb.Xr = at<double>(ar, o_Us64);
    cb.sf2 = f.sf2;
    cb.sn2 = f.sn2;
    cb.band = cov;
    double fl = 0.0;
    if (prof::on)
      for (const BandItem& it : cb_items) fl += 2.0 * it.nr * it.nc * (double)f.s;
    prof::timed(prof::GEMM, fl, st, [&] { launch_band<double>(cb, st); });
    HIPCHK(hipGetLastError());
  }
  auto x_launch = [&](int ci) {
    if (!want_cov) return;
    const int a0 = xsplit[ci], a1 = xsplit[ci + 1];
    if (a1 > a0)
      prof::timed(prof::GEMM, prof::on ? gemm_flops(xterms, xouts, a0, a1) : 0.0, st, [&] {
        launch_tile_gemm<TW>(at<GemmTerm<TW>>(ar, o_xterms), at<GemmOut>(ar, o_xouts) + a0, a1 - a0, st);
      });
    HIPCHK(hipGetLastError());
  };
  if (!var_p) {
    HIPCHK(hipStreamSynchronize(st));
    prof::flush();
    return;
  }
  auto g_launch = [&](int a0, int a1) {
    if (a1 > a0)
      prof::timed(prof::GEMM, prof::on ? gemm_flops(terms, outs, a0, a1) : 0.0, st, [&] { launch_tile_gemm<TW>(at<GemmTerm<TW>>(ar, o_terms), at<GemmOut>(ar, o_outs) + a0, a1 - a0, st); });
    HIPCHK(hipGetLastError());
  };
  auto xi_launch = [&](int64_t m0, int64_t m1, bool accumulate) {
    XiArgs<TW> xa;
    xa.n_u = n_u;
    xa.B = (int)f.B;
    xa.ublk = at<int32_t>(ar, o_ublk);
    xa.uptr = at<int64_t>(ar, o_uptr);
    xa.Xoff = at<int64_t>(ar, o_Xoff);
    xa.Tm = at<int32_t>(ar, o_Tm);
    xa.twm = at<int32_t>(ar, o_twm);
    xa.Xbuf = at<TW>(ar, o_X);
    xa.xi = at<double>(ar, o_xi);
    xa.m0 = (int32_t)m0;
    xa.m1 = (int32_t)m1;
    xa.accumulate = accumulate ? 1 : 0;
    prof::timed(prof::OTHER, 0.0, st, [&] { launch_pred_xi<TW>(xa, st); });
    HIPCHK(hipGetLastError());
  };
  TW* invs = reinterpret_cast<TW*>(f.ptr<char>(f.o_win_inv));
  if (use_tband) {
    BandArgs<TW> ba{};
    ba.items = at<BandItem>(ar, o_tbi);
    ba.nitems = (int32_t)tb_items.size();
    ba.d = (int)d;
    ba.vlen = (int)sp;
    ba.noise = 0;  // test and training points are different sets: no noise term
    ba.vld = sp;
    ba.Vt = f.ptr<double>(f.o_Vt64);
    ba.Xs = f.ptr<double>(f.o_Xs64);
    ba.Vr = at<double>(ar, o_VtU64);
    ba.Xr = at<double>(ar, o_Us64);
    ba.sf2 = f.sf2;
    ba.sn2 = f.sn2;
    ba.band = at<TW>(ar, o_tb);
    double fl = 0.0;
    if (prof::on)
      for (const BandItem& it : tb_items) fl += 2.0 * it.nr * it.nc * (double)f.s;
    prof::timed(prof::GEMM, fl, st, [&] { launch_band<TW>(ba, st); });
    HIPCHK(hipGetLastError());
  }
  if (!stream) {
    exec(runsW[0], invs, (int)sp, false, use_tband);
    for (int dl = 0; dl <= f.B; ++dl) g_launch(dl_split[dl], dl_split[dl + 1]);
    xi_launch(0, M, false);
    x_launch(0);
  } else {
    HIPCHK(hipMemsetAsync(at<double>(ar, o_G), 0, 8 * n_u * ldG, st));
    for (int ci = 0; ci < nch; ++ci) {
      exec(runsW[ci], invs, (int)sp, true);
      for (int dl = 0; dl <= f.B; ++dl) {
        const int k = ci * ((int)f.B + 1) + dl;
        g_launch(gsplit[k], gsplit[k + 1]);
      }
      xi_launch(pchunk[ci], pchunk[ci + 1], ci > 0);
      x_launch(ci);
    }
  }
  PredArgs pa;
  pa.n_u = n_u;
  pa.sp = (int)sp;
  pa.s = (int)f.s;
  pa.d = (int)d;
  pa.G = at<double>(ar, o_G);
  pa.ldG = ldG;
  pa.Us = at<double>(ar, o_Us64);
  pa.Ss = f.ptr<double>(f.o_Ss64);
  pa.VtU = at<double>(ar, o_VtU64);
  pa.g = f.ptr<double>(f.o_g);
  pa.mu = f.mu;
  pa.sf2 = f.sf2;
  pa.sn2 = f.sn2;
  pa.mean = nullptr;
  pa.var = var_p;
  pa.vn = at<double>(ar, o_vn);
  pa.xi = at<double>(ar, o_xi);
  prof::timed(prof::OTHER, 0.0, st, [&] { launch_pred_E(pa, st); });
  HIPCHK(hipGetLastError());
  exec(runD, f.ptr<double>(f.o_Ldd_inv), 0);
  prof::timed(prof::OTHER, 0.0, st, [&] { launch_pred_var(pa, st); });
  HIPCHK(hipGetLastError());
  if (want_cov && !couts.empty()) {
    prof::timed(prof::GEMM, prof::on ? gemm_flops(cterms, couts, 0, (int64_t)couts.size()) : 0.0, st, [&] {
      launch_tile_gemm<double>(at<GemmTerm<double>>(ar, o_cterms), at<GemmOut>(ar, o_couts), (int)couts.size(), st);
    });
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(st));
  prof::flush();
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

lma_status lma_fit(const lma_problem* p, hipStream_t stream, lma_state** out) {
  g_err.clear();
  g_failed = -3;
  if (!out) {
    g_err = "out is NULL";
    return LMA_E_ARG;
  }
  *out = nullptr;
  try {
    return do_fit(p, stream, out, true);
  } catch (const Err& e) {
    set_err(e);
    return e.st;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return LMA_E_NOMEM;
  } catch (const std::exception& e) {
    g_err = std::string("internal error: ") + e.what();
    return LMA_E_INTERNAL;
  }
}

lma_status lma_predict(lma_state* f, int64_t n_u, const double* U, const int64_t* u_block_ptr, double* mean,
                       double* var, hipStream_t stream) {
  g_err.clear();
  g_failed = -3;
  try {
    if (!f) throw Err{LMA_E_ARG, "state is NULL"};
    if (n_u < 0) throw Err{LMA_E_ARG, "n_u < 0"};
    if (n_u == 0) return LMA_OK;
    if (!U || !u_block_ptr || !mean) throw Err{LMA_E_ARG, "NULL array"};
    if (u_block_ptr[0] != 0 || u_block_ptr[f->M] != n_u)
      throw Err{LMA_E_ARG, "u_block_ptr must start at 0 and end at n_u"};
    for (int64_t m = 0; m < f->M; ++m)
      if (u_block_ptr[m + 1] < u_block_ptr[m]) throw Err{LMA_E_ARG, "u_block_ptr must be non-decreasing"};
    if (f->mixed())
      predict_impl<float>(*f, n_u, U, u_block_ptr, mean, var, stream);
    else
      predict_impl<double>(*f, n_u, U, u_block_ptr, mean, var, stream);
    return LMA_OK;
  } catch (const Err& e) {
    set_err(e);
    return e.st;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return LMA_E_NOMEM;
  } catch (const std::exception& e) {
    g_err = std::string("internal error: ") + e.what();
    return LMA_E_INTERNAL;
  }
}

lma_status lma_predict_cov(lma_state* f, int64_t n_u, const double* U, const int64_t* u_block_ptr, double* mean,
                           double* cov, hipStream_t stream) {
  g_err.clear();
  g_failed = -3;
  try {
    if (!f) throw Err{LMA_E_ARG, "state is NULL"};
    if (n_u < 0) throw Err{LMA_E_ARG, "n_u < 0"};
    if (n_u == 0) return LMA_OK;
    if (n_u > ((int64_t)1 << 31)) throw Err{LMA_E_ARG, "n_u too large for a full covariance"};
    if (!U || !u_block_ptr || !cov) throw Err{LMA_E_ARG, "NULL array"};
    if (u_block_ptr[0] != 0 || u_block_ptr[f->M] != n_u)
      throw Err{LMA_E_ARG, "u_block_ptr must start at 0 and end at n_u"};
    for (int64_t m = 0; m < f->M; ++m)
      if (u_block_ptr[m + 1] < u_block_ptr[m]) throw Err{LMA_E_ARG, "u_block_ptr must be non-decreasing"};
    if (f->mixed())
      predict_impl<float>(*f, n_u, U, u_block_ptr, mean, nullptr, stream, cov);
    else
      predict_impl<double>(*f, n_u, U, u_block_ptr, mean, nullptr, stream, cov);
    return LMA_OK;
  } catch (const Err& e) {
    set_err(e);
    return e.st;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return LMA_E_NOMEM;
  } catch (const std::exception& e) {
    g_err = std::string("internal error: ") + e.what();
    return LMA_E_INTERNAL;
  }
}

lma_status lma_lml(const lma_problem* p, double* lml, double* grad, hipStream_t stream) {
  g_err.clear();
  g_failed = -3;
  if (!lml) {
    g_err = "lml is NULL";
    return LMA_E_ARG;
  }
  lma_state* f = nullptr;
  lma_status s = lma_fit(p, stream, &f);
  if (s != LMA_OK) return s;
  std::unique_ptr<lma_state> own(f);
  *lml = f->lml;
  if (!grad) return LMA_OK;
  try {
    // workspace of one chunk of windows: what the budget leaves after the state
    // (at least 256 MB), 16 GB without a budget; LMA_GRAD_CHUNK_BYTES overrides
    int64_t budget = 0;
    if (p->mem_budget_bytes > 0) budget = std::max<int64_t>(p->mem_budget_bytes - f->ar.cap, (int64_t)256 << 20);
    if (const char* e = std::getenv("LMA_GRAD_CHUNK_BYTES")) budget = std::max<long long>(1, std::atoll(e));
    grad_impl(*f, grad, budget, stream);
    return LMA_OK;
  } catch (const Err& e) {
    set_err(e);
    return e.st;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return LMA_E_NOMEM;
  } catch (const std::exception& e) {
    g_err = std::string("internal error: ") + e.what();
    return LMA_E_INTERNAL;
  }
}

lma_status lma_state_lml(const lma_state* f, double* lml) {
  if (!f || !lml) {
    g_err = "NULL argument";
    return LMA_E_ARG;
  }
  *lml = f->lml;
  return LMA_OK;
}

void lma_free(lma_state* f) { delete f; }

int64_t lma_state_bytes(const lma_state* f) { return f ? f->ar.cap : -1; }

int64_t lma_state_chunks(const lma_state* f) { return f ? (int64_t)f->chunk.size() - 1 : -1; }

const char* lma_last_error(void) { return g_err.c_str(); }

int64_t lma_failed_block(void) { return g_failed; }

const char* lma_version(void) { return "lma-gfx950 0.1"; }

void lma_profile_enable(int on) { prof::on = on != 0; }

void lma_release_cache(void) { devcache::release(); }

lma_status lma_profile_read(lma_profile* out, int reset) {
  if (!out) {
    g_err = "out is NULL";
    return LMA_E_ARG;
  }
  *out = prof::acc;
  if (reset) prof::acc = lma_profile{};
  return LMA_OK;
}

}  // extern "C"
