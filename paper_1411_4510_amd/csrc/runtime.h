// Host runtime shared by the fit / predict code and the likelihood gradient:
// error type, device arena and block cache, live timing, the lock-step engine
// schedule (Run), the fitted state and the window geometry helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <string>
#include <type_traits>
#include <vector>

#include "engine.h"
#include "kvec.h"
#include "lma.h"
#include "misc.h"

namespace lmart {
using namespace lma;

struct Err {
  lma_status st;
  std::string msg;
};

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess)                                                                  \
      throw Err{LMA_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)};                \
  } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t align_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// One device allocation per state, carved into 256-byte aligned pieces.
struct Arena {
  char* base = nullptr;
  int64_t cap = 0, used = 0;
  int64_t reserve(int64_t bytes) {
    const int64_t off = used;
    used += align_up(bytes, 256);
    return off;
  }
};

template <typename T>
T* at(const Arena& ar, int64_t off) {
  return reinterpret_cast<T*>(ar.base + off);
}

// Device blocks released by lma_free / lma_predict / the end of a fit are kept
// (at most four) and reused by the next call that fits in them (see lma.hip).
namespace devcache {
void* get(size_t bytes);
void put(void* p, size_t bytes);
void release();
}  // namespace devcache

void ensure_init();
// message returned by lma_last_error() on this thread
void set_last_error(const std::string& msg);

// ---------------------------------------------------------------------------
// live timing: HIP events around launches (enabled by lma_profile_enable)
// ---------------------------------------------------------------------------
namespace prof {
enum Kind { UPDATE = 0, DIAG = 1, TRSM = 2, OTHER = 3, GEMM = 4, CONTRACT = 5 };
extern bool on;
struct Rec {
  int kind;
  hipEvent_t a, b;
  double flops, flops64;
};
extern std::vector<Rec> pending;
extern lma_profile acc;
hipEvent_t get();
template <class F>
void timed(int kind, double flops, hipStream_t st, F&& launch, double flops64 = 0.0) {
  if (!on) {
    launch();
    return;
  }
  Rec r{kind, get(), get(), flops, flops64};
  HIPCHK(hipEventRecord(r.a, st));
  launch();
  HIPCHK(hipEventRecord(r.b, st));
  pending.push_back(r);
}
// call after the stream has been synchronised
void flush();
}  // namespace prof

// 2 x multiply-adds of tile GEMM outputs [o0, o1) on their valid entries
template <typename T>
double gemm_flops(const std::vector<GemmTerm<T>>& terms, const std::vector<GemmOut>& outs, int64_t o0, int64_t o1) {
  double fl = 0.0;
  for (int64_t i = o0; i < o1; ++i) {
    const GemmOut& o = outs[i];
    double k = 0.0;
    for (int t = o.t0; t < o.t1; ++t) k += terms[t].k1 - terms[t].k0;
    fl += 2.0 * o.rows * o.cols * k;
  }
  return fl;
}

// Lock-step column schedule of one engine run, uploaded once.
template <typename T>
struct Run {
  std::vector<ProbDesc> pd;
  std::vector<RowTile<T>> rt;
  std::vector<uint8_t> solve_only;
  std::vector<int32_t> status_block;  // block index reported for each problem
  int maxT = 0;
  // schedule
  std::vector<WorkItem> items;
  std::vector<int32_t> plist;
  std::vector<int64_t> upd_off, upd_n, trs_off, trs_n, pl_off, pl_n;
  // device copies
  RowTile<T>* d_rt = nullptr;
  ProbDesc* d_pd = nullptr;
  WorkItem* d_items = nullptr;
  int32_t* d_plist = nullptr;
  int64_t invdiag_elems = 0;

  int add_problem(int T_, int R, int ld_from, bool so, int block) {
    ProbDesc p;
    p.T = T_;
    p.R = R;
    p.first = (int32_t)rt.size();
    p.ld_from = ld_from;
    p.invdiag_off = invdiag_elems;
    invdiag_elems += (int64_t)T_ * TB * TB;
    pd.push_back(p);
    solve_only.push_back(so ? 1 : 0);
    status_block.push_back(block);
    maxT = std::max(maxT, T_);
    return (int)pd.size() - 1;
  }

  void schedule() {
    const int np = (int)pd.size();
    upd_off.assign(maxT, 0);
    upd_n.assign(maxT, 0);
    trs_off.assign(maxT, 0);
    trs_n.assign(maxT, 0);
    pl_off.assign(maxT, 0);
    pl_n.assign(maxT, 0);
    for (int j = 0; j < maxT; ++j) {
      upd_off[j] = (int64_t)items.size();
      for (int p = 0; p < np; ++p) {
        if (pd[p].T <= j) continue;
        if (!solve_only[p])
          for (int i = j; i < pd[p].T; ++i) items.push_back({p, i});
        for (int r = 0; r < pd[p].R; ++r)
          if (rt[pd[p].first + pd[p].T + r].kbeg <= j) items.push_back({p, pd[p].T + r});
      }
      upd_n[j] = (int64_t)items.size() - upd_off[j];
      trs_off[j] = (int64_t)items.size();
      for (int p = 0; p < np; ++p) {
        if (pd[p].T <= j) continue;
        if (!solve_only[p])
          for (int i = j + 1; i < pd[p].T; ++i) items.push_back({p, i});
        for (int r = 0; r < pd[p].R; ++r)
          if (rt[pd[p].first + pd[p].T + r].kbeg <= j) items.push_back({p, pd[p].T + r});
      }
      trs_n[j] = (int64_t)items.size() - trs_off[j];
      pl_off[j] = (int64_t)plist.size();
      for (int p = 0; p < np; ++p)
        if (pd[p].T > j && !solve_only[p]) plist.push_back(p);
      pl_n[j] = (int64_t)plist.size() - pl_off[j];
    }
  }

  // multiply-adds (x2) of the update launch of step j on real entries only;
  // f64 receives the part done in float64 (all of it for double runs, the V
  // part in mixed runs)
  std::vector<int64_t> cum_nvalid;  // per J tile: real columns before it (built on demand)
  double update_flops(int j, int64_t s_valid, double* f64) {
    if (cum_nvalid.size() != rt.size()) {
      cum_nvalid.assign(rt.size(), 0);
      for (const ProbDesc& p : pd) {
        int64_t acc = 0;
        for (int k = 0; k < p.T; ++k) {
          cum_nvalid[p.first + k] = acc;
          acc += rt[p.first + k].nvalid;
        }
      }
    }
    double f = 0.0, fv = 0.0;
    for (int64_t t = upd_off[j]; t < upd_off[j] + upd_n[j]; ++t) {
      const WorkItem it = items[t];
      const ProbDesc& p = pd[it.p];
      const RowTile<T>& ri = rt[p.first + it.tile];
      const RowTile<T>& rj = rt[p.first + j];
      const double Kv = (ri.vt64 && rj.vt64 && ri.src != SRC_BAND && ri.src != SRC_TBAND) ? (double)s_valid : 0.0;
      const double K = Kv + (double)(cum_nvalid[p.first + j] - cum_nvalid[p.first + std::min(ri.kbeg, j)]);
      const double rows = ri.nvalid, cols = rj.nvalid;
      const double pairs = (ri.is_j && it.tile == j) ? rows * (rows + 1) / 2 : rows * cols;
      f += 2.0 * pairs * K;
      fv += 2.0 * pairs * Kv;
    }
    *f64 = std::is_same<T, double>::value ? f : fv;
    return f;
  }

  int64_t meta_bytes() const {
    return align_up(sizeof(RowTile<T>) * rt.size(), 256) + align_up(sizeof(ProbDesc) * pd.size(), 256) +
           align_up(sizeof(WorkItem) * std::max<size_t>(items.size(), 1), 256) +
           align_up(sizeof(int32_t) * std::max<size_t>(plist.size(), 1), 256);
  }

  void upload(char* dst, hipStream_t st) {
    char* p = dst;
    d_rt = reinterpret_cast<RowTile<T>*>(p);
    if (!rt.empty())
      HIPCHK(hipMemcpyAsync(p, rt.data(), sizeof(RowTile<T>) * rt.size(), hipMemcpyHostToDevice, st));
    p += align_up(sizeof(RowTile<T>) * rt.size(), 256);
    d_pd = reinterpret_cast<ProbDesc*>(p);
    if (!pd.empty())
      HIPCHK(hipMemcpyAsync(p, pd.data(), sizeof(ProbDesc) * pd.size(), hipMemcpyHostToDevice, st));
    p += align_up(sizeof(ProbDesc) * pd.size(), 256);
    d_items = reinterpret_cast<WorkItem*>(p);
    if (!items.empty())
      HIPCHK(hipMemcpyAsync(p, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice, st));
    p += align_up(sizeof(WorkItem) * std::max<size_t>(items.size(), 1), 256);
    d_plist = reinterpret_cast<int32_t*>(p);
    if (!plist.empty())
      HIPCHK(hipMemcpyAsync(p, plist.data(), sizeof(int32_t) * plist.size(), hipMemcpyHostToDevice, st));
  }

};

}  // namespace lmart

// ---------------------------------------------------------------------------
// state
// ---------------------------------------------------------------------------
struct lma_state {
  int precision = 0;
  int64_t n = 0, d = 0, s = 0, M = 0, B = 0, sp = 0, Ts = 0;
  double mu = 0, sf2 = 0, sn2 = 0;
  std::vector<double> log_hyp;
  lma::InvEll ie;
  std::vector<int64_t> bp;
  lmart::Arena ar;
  // offsets in the arena
  int64_t o_Xs64 = -1, o_Ss64 = -1, o_c64 = -1, o_c32 = -1;
  int64_t o_Vt64 = -1, o_Lss = -1, o_Lss_inv = -1;
  int64_t o_win = -1, o_win_inv = -1, o_partial = -1, o_Sdd = -1, o_ydd = -1, o_q = -1;
  int64_t o_Ldd = -1, o_Ldd_inv = -1, o_g = -1, o_logdiag = -1, o_status = -1, o_meta = -1;
  int64_t n_logdiag = 0, n_status = 0;
  // mean path: window table, beta vectors and their V-projections
  int64_t o_wt = -1, o_xJ = -1, o_xW = -1, o_tJ = -1, o_tW = -1, o_hJ = -1, o_hW = -1,
          o_cg = -1, o_dg = -1, o_tvec = -1, o_rho = -1, vec_elems = 0;
  lma::WinTab wt;
  // window geometry
  std::vector<int32_t> Tm, twm;
  std::vector<int64_t> win_off;     // element offset of window m's panels
  std::vector<int64_t> rhs_off;     // element offset of window m's RHS panel (support rows then c row)
  std::vector<int64_t> inv_off;     // element offset of window m's inverted diagonal tiles
  // Window chunks [chunk[c], chunk[c+1]): the windows whose factors are resident
  // together.  One chunk holds all windows unless mem_budget_bytes is too small
  // for that; then win_off / inv_off are relative to the chunk's first window,
  // the window area holds one chunk at a time, and every pass that needs the
  // factors refactors chunk by chunk.
  std::vector<int64_t> chunk;
  int64_t win_area = 0, inv_area = 0;  // elements of the window areas
  std::vector<int64_t> sumsplit;    // summary outputs of chunk c: [sumsplit[c], sumsplit[c+1])
  std::vector<int64_t> kmvsplit;    // KV_KMV items of window m start at kmvsplit[m] ([M+1])
  bool streaming() const { return chunk.size() > 2; }
  int groups = 1, ntile = 1;
  // runs
  lmart::Run<double> runS;
  std::vector<lmart::Run<float>> runsW32;   // window runs, one per chunk
  std::vector<lmart::Run<double>> runsW64;
  lmart::Run<double> runD;
  std::vector<lma::GemmTerm<double>> sum64;
  std::vector<lma::GemmTerm<float>> sum32;
  std::vector<lma::GemmOut> sumout;
  std::vector<int64_t> wt_host;
  int64_t o_sumterms = -1, o_sumout = -1;
  // kernel-times-vector items of the mixed-precision refinement (c' and window residuals)
  std::vector<lma::KvCol> kvcols;
  std::vector<lma::KvItem> kvcg, kvkmv;
  int64_t o_kvcols = -1, o_kvcg = -1, o_kvkmv = -1;
  // results
  std::vector<double> g, ydd;
  double qsum = 0, ld_R = 0, ld_ss = 0, ld_dd = 0, ydg = 0, lml = 0;

  ~lma_state() {
    if (ar.base) lmart::devcache::put(ar.base, (size_t)ar.cap);
  }
  bool mixed() const { return precision == LMA_MIXED; }
  template <typename T>
  T* ptr(int64_t off) const {
    return off < 0 ? nullptr : lmart::at<T>(ar, off);
  }
};

namespace lmart {

// Row-tile panel layout of a problem with T column tiles and R RHS tiles:
// J row tile i holds tiles (i, 0..i) with ld (i+1)*TB; RHS row tile r holds
// tiles (T+r, 0..T-1) with ld T*TB.
inline int64_t jpanel_off(int i) { return (int64_t)TB * TB * i * (i + 1) / 2; }
inline int64_t panel_elems(int T_, int R) { return jpanel_off(T_) + (int64_t)R * TB * T_ * TB; }

template <typename T>
RowTile<T> make_tile(T* panel, int64_t ld, const T* vt, const T* xs, const T* cv, int nvalid, int nstore, int src,
                     int is_j) {
  RowTile<T> r;
  r.panel = panel;
  r.ld = ld;
  r.vt = vt;
  r.xs = xs;
  r.cv = cv;
  r.expl = nullptr;
  r.eld = 0;
  r.nvalid = nvalid;
  r.nstore = nstore;
  r.src = src;
  r.is_j = is_j;
  r.kbeg = 0;
  r.pad_ = 0;
  r.pt0 = 0;
  r.vt64 = std::is_same<T, double>::value ? reinterpret_cast<const double*>(vt) : nullptr;
  r.xs64 = std::is_same<T, double>::value ? reinterpret_cast<const double*>(xs) : nullptr;
  return r;
}

// Window m: W_m = blocks m+1 .. min(m+B, M-1), then D_m.
struct WinGeom {
  int64_t wstart, w, dstart, b;
  int tw, tb, T;
};
inline WinGeom win_geom(const std::vector<int64_t>& bp, int64_t M, int64_t B, int64_t m) {
  WinGeom g;
  const int64_t hi = std::min(m + B, M - 1);
  g.wstart = bp[m + 1 <= M ? m + 1 : M];
  g.w = hi > m ? bp[hi + 1] - bp[m + 1] : 0;
  g.dstart = bp[m];
  g.b = bp[m + 1] - bp[m];
  g.tw = (int)cdiv(g.w, TB);
  g.tb = (int)cdiv(g.b, TB);
  g.T = g.tw + g.tb;
  return g;
}

// First training row and valid rows of J row tile i of a window.
inline int64_t win_tile_point(const WinGeom& g, int i, int* nv) {
  if (i < g.tw) {
    *nv = (int)std::min<int64_t>(TB, g.w - (int64_t)i * TB);
    return g.wstart + (int64_t)i * TB;
  }
  *nv = (int)std::min<int64_t>(TB, g.b - (int64_t)(i - g.tw) * TB);
  return g.dstart + (int64_t)(i - g.tw) * TB;
}

// Column tiles of window m for a kernel-times-vector item: v0 over J_m, v1 over
// W_m (or none).
inline void kv_window_cols(std::vector<KvCol>& cols, const WinGeom& g, const double* Xs, int64_t d, const double* v0,
                           const double* v1) {
  for (int j = 0; j < g.T; ++j) {
    int nv;
    const int64_t p = win_tile_point(g, j, &nv);
    KvCol c;
    c.x = Xs + p * d;
    c.v0 = v0 ? v0 + (int64_t)j * TB : nullptr;
    c.v1 = (v1 && j < g.tw) ? v1 + (int64_t)j * TB : nullptr;
    c.nc = nv;
    c.pad_ = 0;
    cols.push_back(c);
  }
}

inline void kv_support_cols(std::vector<KvCol>& cols, const double* Ss, int64_t s, int64_t d, const double* g) {
  for (int64_t t = 0; t * TB < s; ++t) {
    KvCol c;
    c.x = Ss + t * TB * d;
    c.v0 = g + t * TB;
    c.v1 = nullptr;
    c.nc = (int)std::min<int64_t>(TB, s - t * TB);
    c.pad_ = 0;
    cols.push_back(c);
  }
}

inline KvItem kv_item(const double* x, int nr, int c0, int c1) {
  KvItem it;
  std::memset(&it, 0, sizeof it);
  it.x = x;
  it.nr = nr;
  it.c0 = c0;
  it.c1 = c1;
  return it;
}

// J row tiles of window m (descriptors shared by fit and predict runs).
// Covariance tiles and the V part always read the float64 coordinates and V rows
// (float runs use them through vt64 / xs64 in the mixed update kernel).
template <typename T>
void add_window_jtiles(std::vector<RowTile<T>>& rt, const WinGeom& g, T* base, const double* Xs, const double* Vt,
                       const T* c, int64_t d, int64_t sp, bool band = false) {
  for (int i = 0; i < g.T; ++i) {
    int64_t pt;
    int nv;
    if (i < g.tw) {
      pt = g.wstart + (int64_t)i * TB;
      nv = (int)std::min<int64_t>(TB, g.w - (int64_t)i * TB);
    } else {
      pt = g.dstart + (int64_t)(i - g.tw) * TB;
      nv = (int)std::min<int64_t>(TB, g.b - (int64_t)(i - g.tw) * TB);
    }
    const bool f64 = std::is_same<T, double>::value;
    RowTile<T> t = make_tile<T>(base + jpanel_off(i), (int64_t)(i + 1) * TB,
                                f64 ? reinterpret_cast<const T*>(Vt + pt * sp) : nullptr,
                                f64 ? reinterpret_cast<const T*>(Xs + pt * d) : nullptr, c + pt, nv, TB, SRC_KERNEL, 1);
    t.vt64 = Vt + pt * sp;
    t.xs64 = Xs + pt * d;
    t.pt0 = pt;
    if (band) t.src = SRC_BAND;
    rt.push_back(t);
  }
}

template <typename T>
void add_s_jtiles(std::vector<RowTile<T>>& rt, T* base, const T* Ss, int64_t s, int64_t d, int Ts) {
  for (int i = 0; i < Ts; ++i) {
    const int nv = (int)std::min<int64_t>(TB, s - (int64_t)i * TB);
    rt.push_back(make_tile<T>(base + jpanel_off(i), (int64_t)(i + 1) * TB, nullptr, Ss + (int64_t)i * TB * d,
                              nullptr, nv, TB, SRC_KERNEL, 1));
  }
}

// Inverted diagonal tiles of window m (element offset in the inverse area).
inline int64_t win_inv_off(const lma_state& f, int64_t m) { return f.inv_off[m]; }

// Likelihood gradient of a fitted state (lma_grad.hip): grad[d+2] (host) receives
// d LML / d (log l_1..log l_d, log sigma_s^2, log sigma_n^2).  Windows are
// processed in chunks whose workspace stays under chunk_budget bytes.
void grad_impl(lma_state& f, double* grad, int64_t chunk_budget, hipStream_t st);

}  // namespace lmart
