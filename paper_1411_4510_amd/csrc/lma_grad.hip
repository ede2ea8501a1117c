// Gradient of the LMA log marginal likelihood with respect to
// (log l_1..log l_d, log sigma_s^2, log sigma_n^2), on a fitted state.
//
// The likelihood (whitened window form of Definitions 1-2, Theorem 2 and the
// determinant identity of Lemma 1) depends on the hyperparameters through the
// residual windows R_X (X = J_m with sign +1, X = W_m = D^B_m with sign -1),
// the cross covariances K_XS and Sigma_SS.  Reverse-mode differentiation gives,
// with R_X = L L^T, Y = L^-1 K_XS (the whitened support rows kept by the fit),
// w = R_X^-1 (c_X - K_XS g) (the beta vectors of the mean path), h = V_X w,
// H = Sigma_ddot^-1 and S^-1 = Sigma_SS^-1:
//
//   adjoint of Sigma_XX :  (sign/2) [w w^T - R_X^-1 + Gamma H Gamma^T],  Gamma = R_X^-1 K_XS
//   adjoint of K_XS     :  sign [w u^T + Gamma A_X],  u = g - L_SS^-T h,
//                          A_X = (I - H G0) S^-1 - H,  G0 = Y^T Y
//   adjoint of Sigma_SS :  1/2 [S^-1 - H - g g^T + sum sign hh^T - S^-1 Omega S^-1],
//                          hh = L_SS^-T h, Omega = sum sign (G0 - G0 H G0)
//
// (R_X^-1 enters through an explicit inverse factor X = L^-T computed by the
// engine with identity right-hand sides; for W_m it is the leading block of
// the J_m factor's inverse.)  Each adjoint is contracted tile by tile with the
// derivative of the covariance it multiplies; the covariance tiles are
// regenerated, never stored.  Windows are processed in chunks that fit a
// device-memory budget.
#include <cstdlib>

#include "grad.h"
#include "runtime.h"

namespace lmart {

namespace {

// offset of row panel r of an upper-triangular T x T tile matrix stored by
// rows from its diagonal tile: row r holds tiles r..T-1 (ld (T-r)*TB)
inline int64_t tri_off(int T_, int r) { return (int64_t)TB * TB * ((int64_t)r * T_ - (int64_t)r * (r - 1) / 2); }
inline int64_t tri_elems(int T_) { return (int64_t)TB * TB * T_ * (T_ + 1) / 2; }

template <typename T>
GemmTerm<T> term(const T* a, int64_t lda, int anr, const T* b, int64_t ldb, int bnr, int64_t k1) {
  GemmTerm<T> t;
  t.a = a;
  t.lda = lda;
  t.anr = anr;
  t.b = b;
  t.ldb = ldb;
  t.bnr = bnr;
  t.k0 = 0;
  t.k1 = (int32_t)k1;
  return t;
}

DcItem dc_item(int kind, int nr, int nc, int diag, double wt, const double* xr, const double* xc) {
  DcItem it;
  std::memset(&it, 0, sizeof it);
  it.kind = kind;
  it.nr = nr;
  it.nc = nc;
  it.diag = diag;
  it.wt = wt;
  it.xr = xr;
  it.xc = xc;
  return it;
}
void add_r1(DcItem& it, const double* a, const double* b, double s) {
  it.r1a[it.nr1] = a;
  it.r1b[it.nr1] = b;
  it.r1s[it.nr1] = s;
  ++it.nr1;
}
void add_ex(DcItem& it, const double* e, int64_t ld, double s) {
  it.ex[it.nex] = e;
  it.exld[it.nex] = ld;
  it.exs[it.nex] = s;
  ++it.nex;
}

// Steps of an engine run: solve-only (right-hand sides against stored factors),
// or (factor) factorisation and solves, with the window run's arithmetic; the
// log-diagonals go to ldg[problem * maxT + column].
template <typename TT>
void solve_steps(Run<TT>& run, TT* invdiag, const lma_state& f, double* ldg, int32_t* stat, hipStream_t st,
                 bool factor = false, int maxT = 0) {
  StepArgs<TT> a{};
  a.rt = run.d_rt;
  a.pd = run.d_pd;
  a.vlen = factor ? (int)f.sp : 0;
  a.vld = f.sp;
  a.d = (int)f.d;
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
    const double fl = prof::on ? run.update_flops(j, factor ? f.s : 0, &f64) : 0.0;
    prof::timed(prof::UPDATE, fl, st, [&] { launch_update<TT>(a, factor && std::is_same<TT, float>::value, st); }, f64);
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
}

template <typename T>
void upload_vec(char*& dst, const std::vector<T>& v, hipStream_t st) {
  if (!v.empty()) HIPCHK(hipMemcpyAsync(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
  dst += align_up((int64_t)sizeof(T) * (int64_t)std::max<size_t>(v.size(), 1), 256);
}
template <typename T>
int64_t vec_bytes(const std::vector<T>& v) {
  return align_up((int64_t)sizeof(T) * (int64_t)std::max<size_t>(v.size(), 1), 256);
}


// Host-side bounds check of every operand range the gradient launches will
// touch, against the two device blocks they may live in (the fitted state and
// the gradient workspace).  Throws before anything is launched.
struct Regions {
  const char* lo[3];
  const char* hi[3];
  void need(const void* p, int64_t bytes, const char* what) const {
    const char* c = reinterpret_cast<const char*>(p);
    for (int i = 0; i < 3; ++i)
      if (c >= lo[i] && bytes >= 0 && c + bytes <= hi[i]) return;
    throw Err{LMA_E_ARG, std::string("internal error: gradient operand out of range (") + what + ")"};
  }
  template <typename T>
  void rows(const T* p, int64_t ld, int64_t nrows, int64_t c0, int64_t c1, const char* what) const {
    if (nrows <= 0 || c1 <= c0) return;
    need(p + c0, (int64_t)sizeof(T) * ((nrows - 1) * ld + (c1 - c0)), what);
  }
  template <typename T>
  void gterm(const GemmTerm<T>& t, const char* what) const {
    const int64_t ra = std::max<int64_t>(1, std::min<int64_t>(t.anr, TB));
    const int64_t rb = std::max<int64_t>(1, std::min<int64_t>(t.bnr, TB));
    if (t.k0 % 16 || t.k1 % 16 || t.k1 < t.k0) throw Err{LMA_E_ARG, std::string("internal error: k range (") + what + ")"};
    rows(t.a, t.lda, ra, t.k0, t.k1, what);
    rows(t.b, t.ldb, rb, t.k0, t.k1, what);
  }
  void gout(const GemmOut& o, const char* what) const {
    rows(o.out, o.ld, o.rows, 0, o.cols, what);
    if (o.c) rows(o.c, o.ldc, o.rows, 0, o.cols, what);
  }
};

struct GemmBatch {
  int64_t o0 = 0, o1 = 0;  // outputs [o0, o1)
};

template <typename TW>
void grad_run(lma_state& f, double* grad_host, int64_t budget, hipStream_t st, TW* win_override = nullptr,
              TW* inv_override = nullptr, int64_t override_bytes = 0) {
  const int64_t d = f.d, s = f.s, sp = f.sp, M = f.M;
  const int Ts = (int)f.Ts;
  const int64_t Mp = align_up(M, TB);
  const int64_t sp2 = sp * sp;
  const int ncomp = (int)d + 2;
  const bool mixed = f.mixed();
  TW* winbase = win_override ? win_override : reinterpret_cast<TW*>(f.ptr<char>(f.o_win));
  TW* wininv = inv_override ? inv_override : reinterpret_cast<TW*>(f.ptr<char>(f.o_win_inv));
  const TW* cvec = mixed ? reinterpret_cast<const TW*>(f.ptr<float>(f.o_c32))
                         : reinterpret_cast<const TW*>(f.ptr<double>(f.o_c64));
  const double* Xs = f.ptr<double>(f.o_Xs64);
  const double* Ss = f.ptr<double>(f.o_Ss64);
  const double* Vt = f.ptr<double>(f.o_Vt64);
  const double* xJ = f.ptr<double>(f.o_xJ);
  const double* xW = f.ptr<double>(f.o_xW);

  // ---- chunks of windows
  std::vector<WinGeom> geo(M);
  for (int64_t m = 0; m < M; ++m) geo[m] = win_geom(f.bp, M, f.B, m);
  auto win_bytes = [&](int64_t m) {
    const WinGeom& g = geo[m];
    return (int64_t)sizeof(TW) * tri_elems(g.T) + 8 * (2 * (int64_t)g.T * TB * sp + 2 * (int64_t)g.tw * TB * sp + 8 * sp2);
  };
  std::vector<int64_t> cbeg;  // chunk c = windows [cbeg[c], cbeg[c+1])
  {
    int64_t acc = 0;
    cbeg.push_back(0);
    size_t fc = 1;  // next boundary of the fit's window chunks
    for (int64_t m = 0; m < M; ++m) {
      const int64_t b = win_bytes(m);
      const bool fit_cut = f.streaming() && fc + 1 < f.chunk.size() && m == f.chunk[fc];
      if (fit_cut) ++fc;
      if (acc > 0 && (fit_cut || acc + b > budget)) {
        cbeg.push_back(m);
        acc = 0;
      }
      acc += b;
    }
    cbeg.push_back(M);
  }
  const int nchunk = (int)cbeg.size() - 1;
  // per-window offsets inside the chunk workspace (bytes for X, elements for the rest)
  std::vector<int64_t> xoff(M), goff(M), poff(M), gwoff(M), pwoff(M), soff(M);
  for (int c = 0; c < nchunk; ++c) {
    int64_t xb = 0, de = 0;
    for (int64_t m = cbeg[c]; m < cbeg[c + 1]; ++m) {
      const WinGeom& g = geo[m];
      xoff[m] = xb;
      xb += align_up((int64_t)sizeof(TW) * tri_elems(g.T), 256);
      goff[m] = de;
      de += (int64_t)g.T * TB * sp;
      poff[m] = de;
      de += (int64_t)g.T * TB * sp;
      gwoff[m] = de;
      de += (int64_t)g.tw * TB * sp;
      pwoff[m] = de;
      de += (int64_t)g.tw * TB * sp;
      soff[m] = de;
      de += 8 * sp2;
    }
  }
  int64_t xcap = 0, dcap = 0;
  for (int c = 0; c < nchunk; ++c) {
    int64_t xb = 0, de = 0;
    for (int64_t m = cbeg[c]; m < cbeg[c + 1]; ++m) {
      const WinGeom& g = geo[m];
      xb += align_up((int64_t)sizeof(TW) * tri_elems(g.T), 256);
      de += 2 * (int64_t)g.T * TB * sp + 2 * (int64_t)g.tw * TB * sp + 8 * sp2;
    }
    xcap = std::max(xcap, xb);
    dcap = std::max(dcap, de);
  }
  const int Go = (int)std::max<int64_t>(1, std::min<int64_t>(M, cdiv(512, (int64_t)Ts * Ts)));

  // ---- workspace
  Arena ar;
  const int64_t o_XS = ar.reserve(8 * tri_elems(Ts));
  const int64_t o_Xdd = ar.reserve(8 * tri_elems(Ts));
  const int64_t o_Sinv = ar.reserve(8 * sp2);
  const int64_t o_H = ar.reserve(8 * sp2);
  const int64_t o_D0 = ar.reserve(8 * sp2);
  const int64_t o_SSS = ar.reserve(8 * sp2);
  const int64_t o_Om = ar.reserve(8 * sp2);
  const int64_t o_P = ar.reserve(8 * sp2);
  const int64_t o_HJt = ar.reserve(8 * sp * Mp);
  const int64_t o_HWt = ar.reserve(8 * sp * Mp);
  const int64_t o_uJ = ar.reserve(8 * M * sp);
  const int64_t o_uW = ar.reserve(8 * M * sp);
  const int64_t o_Omp = ar.reserve(8 * (int64_t)Go * sp2);
  const int64_t o_gdev = ar.reserve(8 * ncomp);
  int maxTw = 1;
  for (int64_t m = 0; m < M; ++m) maxTw = std::max(maxTw, (int)f.Tm[m]);
  const int64_t o_stat = ar.reserve(4 * (M + 2));
  const int64_t o_ldg = ar.reserve(8 * (M + 2) * (int64_t)std::max(maxTw, Ts));
  const int64_t o_X = ar.reserve(xcap);
  const int64_t o_D = ar.reserve(8 * dcap);

  // host-side schedules, built against base pointers fixed below
  Run<double> runXS, runXD;
  std::vector<Run<TW>> runX(nchunk);
  std::vector<GemmTerm<TW>> tw_terms;
  std::vector<GemmTerm<double>> d_terms;
  std::vector<GemmOut> outs_tw, outs_d;
  std::vector<DcItem> items;
  std::vector<GemmTerm<TW>> x_terms;
  GemmBatch prepB, finB;
  std::vector<GemmBatch> c2(nchunk), c2b(nchunk), c3(nchunk), c4(nchunk);
  std::vector<int64_t> it_beg(nchunk + 2);

  auto build = [&](char* base) {
    ar.base = base;
    runXS = Run<double>();
    runXD = Run<double>();
    for (auto& r : runX) r = Run<TW>();
    tw_terms.clear();
    d_terms.clear();
    outs_tw.clear();
    outs_d.clear();
    items.clear();
    x_terms.clear();
    double* XS = at<double>(ar, o_XS);
    double* Xdd = at<double>(ar, o_Xdd);
    double* Sinv = at<double>(ar, o_Sinv);
    double* H = at<double>(ar, o_H);
    double* D0 = at<double>(ar, o_D0);
    double* Om = at<double>(ar, o_Om);
    double* P = at<double>(ar, o_P);
    double* HJt = at<double>(ar, o_HJt);
    double* HWt = at<double>(ar, o_HWt);
    double* uJ = at<double>(ar, o_uJ);
    double* uW = at<double>(ar, o_uW);
    double* Omp = at<double>(ar, o_Omp);
    TW* Xb = reinterpret_cast<TW*>(at<char>(ar, o_X));
    double* Db = at<double>(ar, o_D);
    const double* hJ = f.ptr<double>(f.o_hJ);
    const double* hW = f.ptr<double>(f.o_hW);

    // identity solves on Sigma_SS and Sigma_ddot: rows of L_SS^-T and L_ddot^-T
    auto ident_rows = [&](Run<double>& run, double* Xt) {
      for (int r = 0; r < Ts; ++r) {
        RowTile<double> t = make_tile<double>(Xt + tri_off(Ts, r), (int64_t)(Ts - r) * TB, nullptr, nullptr, nullptr,
                                              TB, TB, SRC_IDENT, 0);
        t.kbeg = r;
        run.rt.push_back(t);
      }
    };
    runXS.add_problem(Ts, Ts, 0, true, -1);
    add_s_jtiles<double>(runXS.rt, f.ptr<double>(f.o_Lss), Ss, s, d, Ts);
    ident_rows(runXS, XS);
    runXS.schedule();
    runXD.add_problem(Ts, Ts, 0, true, -2);
    for (int i = 0; i < Ts; ++i)
      runXD.rt.push_back(make_tile<double>(f.ptr<double>(f.o_Ldd) + jpanel_off(i), (int64_t)(i + 1) * TB, nullptr,
                                           nullptr, nullptr, (int)std::min<int64_t>(TB, s - (int64_t)i * TB), TB,
                                           SRC_EXPLICIT, 1));
    ident_rows(runXD, Xdd);
    runXD.schedule();

    // prep products: S^-1 = X_S X_S^T, H = X_dd X_dd^T, hh^T = X_S h^T
    prepB.o0 = (int64_t)outs_d.size();
    for (int pa = 0; pa < Ts; ++pa)
      for (int pb = 0; pb < Ts; ++pb) {
        const int kk = std::max(pa, pb);
        for (int w = 0; w < 2; ++w) {
          double* Xt = w ? Xdd : XS;
          GemmOut o = gemm_out((w ? H : Sinv) + (int64_t)pa * TB * sp + (int64_t)pb * TB, sp, TB, TB, 0,
                               (int)d_terms.size());
          d_terms.push_back(term<double>(Xt + tri_off(Ts, pa) + (int64_t)(kk - pa) * TB, (int64_t)(Ts - pa) * TB, TB,
                                         Xt + tri_off(Ts, pb) + (int64_t)(kk - pb) * TB, (int64_t)(Ts - pb) * TB, TB,
                                         (int64_t)(Ts - kk) * TB));
          o.t1 = (int32_t)d_terms.size();
          outs_d.push_back(o);
        }
      }
    for (int t = 0; t < Ts; ++t)
      for (int64_t xt = 0; xt < Mp / TB; ++xt) {
        const int cols = (int)std::min<int64_t>(TB, M - xt * TB);
        for (int w = 0; w < 2; ++w) {
          GemmOut o = gemm_out((w ? HWt : HJt) + (int64_t)t * TB * Mp + xt * TB, Mp, TB, cols, 0, (int)d_terms.size());
          d_terms.push_back(term<double>(XS + tri_off(Ts, t), (int64_t)(Ts - t) * TB, TB,
                                         (w ? hW : hJ) + xt * TB * sp + (int64_t)t * TB, sp, cols,
                                         (int64_t)(Ts - t) * TB));
          o.t1 = (int32_t)d_terms.size();
          outs_d.push_back(o);
        }
      }
    prepB.o1 = (int64_t)outs_d.size();

    // per chunk
    for (int c = 0; c < nchunk; ++c) {
      Run<TW>& run = runX[c];
      for (int64_t m = cbeg[c]; m < cbeg[c + 1]; ++m) {
        const WinGeom& g = geo[m];
        // factors held one chunk at a time: factor the window again, with its
        // support rows and output row, before the identity rows
        const bool refactor = f.streaming();
        run.add_problem(g.T, g.T + (refactor ? Ts + 1 : 0), g.tw, !refactor, (int)m);
        add_window_jtiles<TW>(run.rt, g, winbase + f.win_off[m], Xs, Vt, cvec, d, sp);
        run.pd.back().invdiag_off = win_inv_off(f, m);
        if (refactor) {
          TW* rhs = winbase + f.win_off[m] + jpanel_off(g.T);
          const int64_t ldr = (int64_t)g.T * TB;
          for (int r = 0; r < Ts; ++r) {
            const int nv = (int)std::min<int64_t>(TB, s - (int64_t)r * TB);
            const bool f64 = std::is_same<TW, double>::value;
            RowTile<TW> t = make_tile<TW>(rhs + (int64_t)r * TB * ldr, ldr, nullptr,
                                          f64 ? reinterpret_cast<const TW*>(Ss + (int64_t)r * TB * d) : nullptr,
                                          nullptr, nv, TB, SRC_KERNEL, 0);
            t.xs64 = Ss + (int64_t)r * TB * d;
            run.rt.push_back(t);
          }
          run.rt.push_back(make_tile<TW>(rhs + (int64_t)Ts * TB * ldr, ldr, nullptr, nullptr, nullptr, 1, TB, SRC_CVEC, 0));
        }
        TW* Xm = reinterpret_cast<TW*>(reinterpret_cast<char*>(Xb) + xoff[m]);
        for (int r = 0; r < g.T; ++r) {
          RowTile<TW> t = make_tile<TW>(Xm + tri_off(g.T, r), (int64_t)(g.T - r) * TB, nullptr, nullptr, nullptr, TB,
                                        TB, SRC_IDENT, 0);
          t.kbeg = r;
          run.rt.push_back(t);
        }
      }
      run.schedule();
      // Gamma_W = X_W Y_W and G0_W = Y_W^T Y_W first.  X_W and Y_W are the leading
      // blocks of X_J and Y_J (W_m leads the window order), so the J products then
      // reuse them: Gamma_J rows i < tw = Gamma_W + X[i, tw:T] Y[tw:T] and
      // G0_J = G0_W + Y_D^T Y_D.
      c2[c].o0 = (int64_t)outs_tw.size();
      for (int64_t m = cbeg[c]; m < cbeg[c + 1]; ++m) {
        const WinGeom& g = geo[m];
        const TW* Xm = reinterpret_cast<const TW*>(reinterpret_cast<char*>(Xb) + xoff[m]);
        const TW* R = winbase + f.win_off[m] + jpanel_off(g.T);
        const int64_t ldR = (int64_t)g.T * TB;
        double* GW = Db + gwoff[m];
        double* G0W = Db + soff[m] + sp2;
        for (int i = 0; i < g.tw; ++i)
          for (int t = 0; t < Ts; ++t) {
            GemmOut o = gemm_out(GW + (int64_t)i * TB * sp + (int64_t)t * TB, sp, TB, TB, 0, (int)tw_terms.size());
            tw_terms.push_back(term<TW>(Xm + tri_off(g.T, i), (int64_t)(g.T - i) * TB, TB,
                                        R + (int64_t)t * TB * ldR + (int64_t)i * TB, ldR, TB,
                                        (int64_t)(g.tw - i) * TB));
            o.t1 = (int32_t)tw_terms.size();
            outs_tw.push_back(o);
          }
        if (g.tw > 0)
          for (int pa = 0; pa < Ts; ++pa)
            for (int pb = 0; pb < Ts; ++pb) {
              GemmOut o = gemm_out(G0W + (int64_t)pa * TB * sp + (int64_t)pb * TB, sp, TB, TB, 0, (int)tw_terms.size());
              tw_terms.push_back(term<TW>(R + (int64_t)pa * TB * ldR, ldR, TB, R + (int64_t)pb * TB * ldR, ldR, TB,
                                          (int64_t)g.tw * TB));
              o.t1 = (int32_t)tw_terms.size();
              outs_tw.push_back(o);
            }
      }
      c2[c].o1 = (int64_t)outs_tw.size();
      c2b[c].o0 = (int64_t)outs_tw.size();
      for (int64_t m = cbeg[c]; m < cbeg[c + 1]; ++m) {
        const WinGeom& g = geo[m];
        const TW* Xm = reinterpret_cast<const TW*>(reinterpret_cast<char*>(Xb) + xoff[m]);
        const TW* R = winbase + f.win_off[m] + jpanel_off(g.T);
        const int64_t ldR = (int64_t)g.T * TB;
        double* GJ = Db + goff[m];
        const double* GW = Db + gwoff[m];
        double* G0J = Db + soff[m];
        const double* G0W = G0J + sp2;
        for (int i = 0; i < g.T; ++i)
          for (int t = 0; t < Ts; ++t) {
            const int k0 = i < g.tw ? g.tw : i;  // first column of X row i still to add
            GemmOut o = gemm_out(GJ + (int64_t)i * TB * sp + (int64_t)t * TB, sp, TB, TB, 0, (int)tw_terms.size());
            if (i < g.tw) {
              o.c = GW + (int64_t)i * TB * sp + (int64_t)t * TB;
              o.ldc = sp;
              o.beta = 1.0;
            }
            tw_terms.push_back(term<TW>(Xm + tri_off(g.T, i) + (int64_t)(k0 - i) * TB, (int64_t)(g.T - i) * TB, TB,
                                        R + (int64_t)t * TB * ldR + (int64_t)k0 * TB, ldR, TB,
                                        (int64_t)(g.T - k0) * TB));
            o.t1 = (int32_t)tw_terms.size();
            outs_tw.push_back(o);
          }
        for (int pa = 0; pa < Ts; ++pa)
          for (int pb = 0; pb < Ts; ++pb) {
            GemmOut o = gemm_out(G0J + (int64_t)pa * TB * sp + (int64_t)pb * TB, sp, TB, TB, 0, (int)tw_terms.size());
            if (g.tw > 0) {
              o.c = G0W + (int64_t)pa * TB * sp + (int64_t)pb * TB;
              o.ldc = sp;
              o.beta = 1.0;
            }
            tw_terms.push_back(term<TW>(R + (int64_t)pa * TB * ldR + (int64_t)g.tw * TB, ldR, TB,
                                        R + (int64_t)pb * TB * ldR + (int64_t)g.tw * TB, ldR, TB,
                                        (int64_t)(g.T - g.tw) * TB));
            o.t1 = (int32_t)tw_terms.size();
            outs_tw.push_back(o);
          }
      }
      c2b[c].o1 = (int64_t)outs_tw.size();
      // Phi = Gamma H, Xi = G0 H, Ups = H G0
      c3[c].o0 = (int64_t)outs_d.size();
      for (int64_t m = cbeg[c]; m < cbeg[c + 1]; ++m) {
        const WinGeom& g = geo[m];
        for (int w = 0; w < 2; ++w) {
          const int rows_t = w ? g.tw : g.T;
          double* Gm = Db + (w ? gwoff[m] : goff[m]);
          double* Pm = Db + (w ? pwoff[m] : poff[m]);
          for (int i = 0; i < rows_t; ++i)
            for (int t = 0; t < Ts; ++t) {
              GemmOut o = gemm_out(Pm + (int64_t)i * TB * sp + (int64_t)t * TB, sp, TB, TB, 0, (int)d_terms.size());
              d_terms.push_back(term<double>(Gm + (int64_t)i * TB * sp, sp, TB, H + (int64_t)t * TB * sp, sp, TB, sp));
              o.t1 = (int32_t)d_terms.size();
              outs_d.push_back(o);
            }
          if (rows_t == 0) continue;
          double* G0 = Db + soff[m] + (int64_t)w * sp2;
          double* Xi = Db + soff[m] + (int64_t)(2 + w) * sp2;
          double* Up = Db + soff[m] + (int64_t)(4 + w) * sp2;
          for (int pa = 0; pa < Ts; ++pa)
            for (int pb = 0; pb < Ts; ++pb) {
              GemmOut o = gemm_out(Xi + (int64_t)pa * TB * sp + (int64_t)pb * TB, sp, TB, TB, 0, (int)d_terms.size());
              d_terms.push_back(term<double>(G0 + (int64_t)pa * TB * sp, sp, TB, H + (int64_t)pb * TB * sp, sp, TB, sp));
              o.t1 = (int32_t)d_terms.size();
              outs_d.push_back(o);
              GemmOut o2 = gemm_out(Up + (int64_t)pa * TB * sp + (int64_t)pb * TB, sp, TB, TB, 0, (int)d_terms.size());
              d_terms.push_back(term<double>(H + (int64_t)pa * TB * sp, sp, TB, G0 + (int64_t)pb * TB * sp, sp, TB, sp));
              o2.t1 = (int32_t)d_terms.size();
              outs_d.push_back(o2);
            }
        }
      }
      c3[c].o1 = (int64_t)outs_d.size();
      // A_X^T = D0 - S^-1 Xi_X ; Omega partials += Xi_W G0_W - Xi_J G0_J
      c4[c].o0 = (int64_t)outs_d.size();
      for (int64_t m = cbeg[c]; m < cbeg[c + 1]; ++m) {
        const WinGeom& g = geo[m];
        for (int w = 0; w < 2; ++w) {
          if ((w ? g.tw : g.T) == 0) continue;
          double* Up = Db + soff[m] + (int64_t)(4 + w) * sp2;
          double* Am = Db + soff[m] + (int64_t)(6 + w) * sp2;
          for (int pa = 0; pa < Ts; ++pa)
            for (int pb = 0; pb < Ts; ++pb) {
              GemmOut o = gemm_out(Am + (int64_t)pa * TB * sp + (int64_t)pb * TB, sp, TB, TB, 0, (int)d_terms.size());
              d_terms.push_back(term<double>(Sinv + (int64_t)pa * TB * sp, sp, TB, Up + (int64_t)pb * TB * sp, sp, TB, sp));
              o.t1 = (int32_t)d_terms.size();
              o.alpha = -1.0;
              o.c = D0 + (int64_t)pa * TB * sp + (int64_t)pb * TB;
              o.ldc = sp;
              o.beta = 1.0;
              outs_d.push_back(o);
            }
        }
      }
      for (int gi = 0; gi < Go; ++gi) {
        std::vector<int64_t> ms;
        for (int64_t m = cbeg[c]; m < cbeg[c + 1]; ++m)
          if (m % Go == gi) ms.push_back(m);
        if (ms.empty()) continue;
        for (int pa = 0; pa < Ts; ++pa)
          for (int pb = 0; pb < Ts; ++pb) {
            GemmOut o = gemm_out(Omp + (int64_t)gi * sp2 + (int64_t)pa * TB * sp + (int64_t)pb * TB, sp, TB, TB, 1,
                                 (int)d_terms.size());
            for (int w = 0; w < 2; ++w) {  // J terms subtracted first, then W terms added
              if (w == 1) o.tneg = (int32_t)d_terms.size();
              for (int64_t m : ms) {
                if ((w ? geo[m].tw : geo[m].T) == 0) continue;
                const double* G0 = Db + soff[m] + (int64_t)w * sp2;
                const double* Xi = Db + soff[m] + (int64_t)(2 + w) * sp2;
                d_terms.push_back(term<double>(Xi + (int64_t)pa * TB * sp, sp, TB, G0 + (int64_t)pb * TB * sp, sp, TB, sp));
              }
            }
            o.t1 = (int32_t)d_terms.size();
            outs_d.push_back(o);
          }
      }
      c4[c].o1 = (int64_t)outs_d.size();
      // contraction items: residual-window adjoints, then K_XS adjoints
      it_beg[c] = (int64_t)items.size();
      for (int64_t m = cbeg[c]; m < cbeg[c + 1]; ++m) {
        const WinGeom& g = geo[m];
        const TW* Xm = reinterpret_cast<const TW*>(reinterpret_cast<char*>(Xb) + xoff[m]);
        const int64_t vo = f.wt_host[6 * M + m];
        auto tile_pts = [&](int i, int& nv) -> int64_t {
          if (i < g.tw) {
            nv = (int)std::min<int64_t>(TB, g.w - (int64_t)i * TB);
            return g.wstart + (int64_t)i * TB;
          }
          nv = (int)std::min<int64_t>(TB, g.b - (int64_t)(i - g.tw) * TB);
          return g.dstart + (int64_t)(i - g.tw) * TB;
        };
        const double* GJ = Db + goff[m];
        const double* PJ = Db + poff[m];
        const double* GW = Db + gwoff[m];
        const double* PW = Db + pwoff[m];
        for (int i = 0; i < g.T; ++i) {
          int nri;
          const int64_t pi = tile_pts(i, nri);
          for (int j = 0; j <= i; ++j) {
            int ncj;
            const int64_t pj = tile_pts(j, ncj);
            DcItem it = dc_item(DC_SAME, nri, ncj, i == j, i == j ? 0.5 : 1.0, Xs + pi * d, Xs + pj * d);
            const int kk = std::max(g.tw, i);
            it.x0 = (int32_t)x_terms.size();
            if (kk < g.T)
              x_terms.push_back(term<TW>(Xm + tri_off(g.T, i) + (int64_t)(kk - i) * TB, (int64_t)(g.T - i) * TB, TB,
                                         Xm + tri_off(g.T, j) + (int64_t)(kk - j) * TB, (int64_t)(g.T - j) * TB, TB,
                                         (int64_t)(g.T - kk) * TB));
            it.x1 = (int32_t)x_terms.size();
            it.t0 = (int32_t)d_terms.size();
            if (i < g.tw)
              d_terms.push_back(term<double>(PW + (int64_t)i * TB * sp, sp, TB, GW + (int64_t)j * TB * sp, sp, TB, sp));
            it.tneg = (int32_t)d_terms.size();
            d_terms.push_back(term<double>(PJ + (int64_t)i * TB * sp, sp, TB, GJ + (int64_t)j * TB * sp, sp, TB, sp));
            it.t1 = (int32_t)d_terms.size();
            add_r1(it, xJ + vo + (int64_t)i * TB, xJ + vo + (int64_t)j * TB, 1.0);
            if (i < g.tw) add_r1(it, xW + vo + (int64_t)i * TB, xW + vo + (int64_t)j * TB, -1.0);
            items.push_back(it);
          }
        }
        const double* AJ = Db + soff[m] + 6 * sp2;
        const double* AW = Db + soff[m] + 7 * sp2;
        for (int i = 0; i < g.T; ++i) {
          int nri;
          const int64_t pi = tile_pts(i, nri);
          for (int t = 0; t < Ts; ++t) {
            const int nct = (int)std::min<int64_t>(TB, s - (int64_t)t * TB);
            DcItem it = dc_item(DC_CROSS, nri, nct, 0, 1.0, Xs + pi * d, Ss + (int64_t)t * TB * d);
            it.x0 = it.x1 = (int32_t)x_terms.size();
            it.t0 = (int32_t)d_terms.size();
            if (i < g.tw)
              d_terms.push_back(term<double>(GW + (int64_t)i * TB * sp, sp, TB, AW + (int64_t)t * TB * sp, sp, TB, sp));
            it.tneg = (int32_t)d_terms.size();
            d_terms.push_back(term<double>(GJ + (int64_t)i * TB * sp, sp, TB, AJ + (int64_t)t * TB * sp, sp, TB, sp));
            it.t1 = (int32_t)d_terms.size();
            add_r1(it, xJ + vo + (int64_t)i * TB, uJ + m * sp + (int64_t)t * TB, 1.0);
            if (i < g.tw) add_r1(it, xW + vo + (int64_t)i * TB, uW + m * sp + (int64_t)t * TB, -1.0);
            items.push_back(it);
          }
        }
      }
    }
    it_beg[nchunk] = (int64_t)items.size();
    // final: P = S^-1 Omega, then the Sigma_SS adjoint
    finB.o0 = (int64_t)outs_d.size();
    for (int pa = 0; pa < Ts; ++pa)
      for (int pb = 0; pb < Ts; ++pb) {
        GemmOut o = gemm_out(P + (int64_t)pa * TB * sp + (int64_t)pb * TB, sp, TB, TB, 0, (int)d_terms.size());
        d_terms.push_back(term<double>(Sinv + (int64_t)pa * TB * sp, sp, TB, Om + (int64_t)pb * TB * sp, sp, TB, sp));
        o.t1 = (int32_t)d_terms.size();
        outs_d.push_back(o);
      }
    finB.o1 = (int64_t)outs_d.size();
    const double* g = f.ptr<double>(f.o_g);
    for (int pa = 0; pa < Ts; ++pa)
      for (int pb = 0; pb < Ts; ++pb) {
        const int na = (int)std::min<int64_t>(TB, s - (int64_t)pa * TB);
        const int nb = (int)std::min<int64_t>(TB, s - (int64_t)pb * TB);
        DcItem it = dc_item(DC_SAME, na, nb, pa == pb, 0.5, Ss + (int64_t)pa * TB * d, Ss + (int64_t)pb * TB * d);
        it.x0 = it.x1 = (int32_t)x_terms.size();
        it.t0 = (int32_t)d_terms.size();
        d_terms.push_back(term<double>(P + (int64_t)pa * TB * sp, sp, TB, Sinv + (int64_t)pb * TB * sp, sp, TB, sp));
        d_terms.push_back(term<double>(HWt + (int64_t)pa * TB * Mp, Mp, TB, HWt + (int64_t)pb * TB * Mp, Mp, TB, Mp));
        it.tneg = (int32_t)d_terms.size();
        d_terms.push_back(term<double>(HJt + (int64_t)pa * TB * Mp, Mp, TB, HJt + (int64_t)pb * TB * Mp, Mp, TB, Mp));
        it.t1 = (int32_t)d_terms.size();
        add_ex(it, Sinv + (int64_t)pa * TB * sp + (int64_t)pb * TB, sp, 1.0);
        add_ex(it, H + (int64_t)pa * TB * sp + (int64_t)pb * TB, sp, -1.0);
        add_r1(it, g + (int64_t)pa * TB, g + (int64_t)pb * TB, -1.0);
        items.push_back(it);
      }
    it_beg[nchunk + 1] = (int64_t)items.size();
  };
  build(nullptr);
  int64_t meta = runXS.meta_bytes() + runXD.meta_bytes();
  for (auto& r : runX) meta += r.meta_bytes();
  meta += vec_bytes(tw_terms) + vec_bytes(d_terms) + vec_bytes(outs_tw) + vec_bytes(outs_d) + vec_bytes(items) +
          vec_bytes(x_terms);
  const int64_t nitems = (int64_t)items.size();
  const int64_t o_part = ar.reserve(8 * nitems * ncomp);
  const int64_t o_meta = ar.reserve(meta);
  ar.cap = ar.used;
  void* mem = devcache::get((size_t)ar.cap);
  if (!mem) throw Err{LMA_E_NOMEM, "device allocation of the gradient workspace failed"};
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
    Regions rg;
    rg.lo[0] = f.ar.base;
    rg.hi[0] = f.ar.base + f.ar.cap;
    rg.lo[1] = reinterpret_cast<const char*>(mem);
    rg.hi[1] = reinterpret_cast<const char*>(mem) + ar.cap;
    rg.lo[2] = rg.hi[2] = nullptr;
    if (win_override) {
      rg.lo[2] = reinterpret_cast<const char*>(win_override);
      rg.hi[2] = rg.lo[2] + override_bytes;
    }
    for (const GemmTerm<TW>& t : tw_terms) rg.gterm(t, "window product term");
    for (const GemmTerm<double>& t : d_terms) rg.gterm(t, "float64 product term");
    for (const GemmTerm<TW>& t : x_terms) rg.gterm(t, "inverse-factor term");
    for (const GemmOut& o : outs_tw) {
      rg.gout(o, "window product output");
      for (int t = o.t0; t < o.t1; ++t)
        if (o.rows > tw_terms[t].anr || o.cols > tw_terms[t].bnr) throw Err{LMA_E_ARG, "internal error: output rows"};
    }
    for (const GemmOut& o : outs_d) {
      rg.gout(o, "float64 product output");
      for (int t = o.t0; t < o.t1; ++t)
        if (o.rows > d_terms[t].anr || o.cols > d_terms[t].bnr) throw Err{LMA_E_ARG, "internal error: output rows"};
    }
    for (const DcItem& it : items) {
      rg.rows(it.xr, d, it.nr, 0, d, "row coordinates");
      rg.rows(it.xc, d, it.nc, 0, d, "column coordinates");
      for (int r = 0; r < it.nr1; ++r) {
        rg.rows(it.r1a[r], 1, 1, 0, it.nr, "rank-one rows");
        rg.rows(it.r1b[r], 1, 1, 0, it.nc, "rank-one columns");
      }
      for (int x = 0; x < it.nex; ++x) rg.rows(it.ex[x], it.exld[x], it.nr, 0, it.nc, "explicit term");
      if (it.x1 > (int)x_terms.size() || it.t1 > (int)d_terms.size()) throw Err{LMA_E_ARG, "internal error: terms"};
      for (int t = it.x0; t < it.x1; ++t)
        if (it.nr > x_terms[t].anr || it.nc > x_terms[t].bnr) throw Err{LMA_E_ARG, "internal error: item rows"};
      for (int t = it.t0; t < it.t1; ++t)
        if (it.nr > d_terms[t].anr || it.nc > d_terms[t].bnr) throw Err{LMA_E_ARG, "internal error: item rows"};
    }
    auto check_run = [&](auto& run) {
      for (const ProbDesc& pdsc : run.pd)
        for (int r = 0; r < pdsc.R; ++r) {
          const auto& t = run.rt[pdsc.first + pdsc.T + r];
          rg.rows(t.panel, t.ld, t.nstore, 0, (int64_t)(pdsc.T - t.kbeg) * TB, "inverse-factor rows");
        }
    };
    check_run(runXS);
    check_run(runXD);
    for (auto& r : runX) check_run(r);
  }
  // upload schedules
  char* mp = at<char>(ar, o_meta);
  runXS.upload(mp, st);
  mp += runXS.meta_bytes();
  runXD.upload(mp, st);
  mp += runXD.meta_bytes();
  for (auto& r : runX) {
    r.upload(mp, st);
    mp += r.meta_bytes();
  }
  const GemmTerm<TW>* dtw_terms = reinterpret_cast<const GemmTerm<TW>*>(mp);
  upload_vec(mp, tw_terms, st);
  const GemmTerm<double>* dd_terms = reinterpret_cast<const GemmTerm<double>*>(mp);
  upload_vec(mp, d_terms, st);
  const GemmOut* douts_tw = reinterpret_cast<const GemmOut*>(mp);
  upload_vec(mp, outs_tw, st);
  const GemmOut* douts_d = reinterpret_cast<const GemmOut*>(mp);
  upload_vec(mp, outs_d, st);
  const DcItem* ditems = reinterpret_cast<const DcItem*>(mp);
  upload_vec(mp, items, st);
  const GemmTerm<TW>* dx_terms = reinterpret_cast<const GemmTerm<TW>*>(mp);
  upload_vec(mp, x_terms, st);

  double* part = at<double>(ar, o_part);
  int32_t* stat = at<int32_t>(ar, o_stat);
  double* ldg = at<double>(ar, o_ldg);
  auto gemm_d = [&](const GemmBatch& b) {
    if (b.o1 > b.o0)
      prof::timed(prof::GEMM, prof::on ? gemm_flops(d_terms, outs_d, b.o0, b.o1) : 0.0, st,
                  [&] { launch_tile_gemm<double>(dd_terms, douts_d + b.o0, (int)(b.o1 - b.o0), st); });
    HIPCHK(hipGetLastError());
  };
  // 2 x multiply-adds of the tile products of contraction items [i0, i1) on valid entries
  auto contract_flops = [&](int64_t i0, int64_t i1) {
    double fl = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
      const DcItem& it = items[i];
      double k = 0.0;
      for (int t = it.x0; t < it.x1; ++t) k += x_terms[t].k1 - x_terms[t].k0;
      for (int t = it.t0; t < it.t1; ++t) k += d_terms[t].k1 - d_terms[t].k0;
      fl += 2.0 * it.nr * it.nc * k;
    }
    return fl;
  };
  auto contract = [&](int64_t i0, int64_t i1) {
    DcArgs<TW> a;
    a.items = ditems + i0;
    a.nitems = (int32_t)(i1 - i0);
    a.d = (int)d;
    a.xterms = dx_terms;
    a.terms = dd_terms;
    a.sf2 = f.sf2;
    a.sn2 = f.sn2;
    a.partial = part + i0 * ncomp;
    if (i1 > i0)
      prof::timed(prof::CONTRACT, prof::on ? contract_flops(i0, i1) : 0.0, st, [&] { launch_dcontract<TW>(a, st); });
    HIPCHK(hipGetLastError());
  };

  // ---- prep
  prof::timed(prof::OTHER, 0.0, st, [&] { launch_zero(at<double>(ar, o_Omp), (int64_t)Go * sp2, st); });
  prof::timed(prof::OTHER, 0.0, st, [&] { launch_zero(at<double>(ar, o_HJt), sp * Mp, st); });
  prof::timed(prof::OTHER, 0.0, st, [&] { launch_zero(at<double>(ar, o_HWt), sp * Mp, st); });
  solve_steps<double>(runXS, f.ptr<double>(f.o_Lss_inv), f, ldg, stat, st);
  solve_steps<double>(runXD, f.ptr<double>(f.o_Ldd_inv), f, ldg, stat, st);
  gemm_d(prepB);
  prof::timed(prof::OTHER, 0.0, st, [&] {
    launch_lincomb(at<double>(ar, o_D0), at<double>(ar, o_Sinv), 1.0, at<double>(ar, o_H), -1.0, sp2, st);
  });
  prof::timed(prof::OTHER, 0.0, st, [&] { launch_sig_ss(Ss, (int)s, (int)sp, (int)d, f.sf2, f.sn2, at<double>(ar, o_SSS), st); });
  prof::timed(prof::OTHER, 0.0, st, [&] {
    launch_uvec(at<double>(ar, o_uJ), f.ptr<double>(f.o_g), at<double>(ar, o_HJt), Mp, (int)M, (int)sp, st);
  });
  prof::timed(prof::OTHER, 0.0, st, [&] {
    launch_uvec(at<double>(ar, o_uW), f.ptr<double>(f.o_g), at<double>(ar, o_HWt), Mp, (int)M, (int)sp, st);
  });
  HIPCHK(hipGetLastError());
  // ---- window chunks
  for (int c = 0; c < nchunk; ++c) {
    solve_steps<TW>(runX[c], wininv, f, ldg, stat, st, f.streaming(), maxTw);
    for (const GemmBatch& b : {c2[c], c2b[c]})
      if (b.o1 > b.o0)
        prof::timed(prof::GEMM, prof::on ? gemm_flops(tw_terms, outs_tw, b.o0, b.o1) : 0.0, st, [&] {
          launch_tile_gemm<TW>(dtw_terms, douts_tw + b.o0, (int)(b.o1 - b.o0), st);
        });
    HIPCHK(hipGetLastError());
    gemm_d(c3[c]);
    gemm_d(c4[c]);
    contract(it_beg[c], it_beg[c + 1]);
  }
  // ---- Sigma_SS adjoint
  prof::timed(prof::OTHER, 0.0, st, [&] {
    launch_sum_groups(at<double>(ar, o_Om), f.ptr<double>(f.o_Sdd), at<double>(ar, o_SSS), at<double>(ar, o_Omp), Go,
                      sp2, st);
  });
  gemm_d(finB);
  contract(it_beg[nchunk], it_beg[nchunk + 1]);
  if (std::getenv("LMA_GRAD_PARTS")) {  // diagnostic: sums of the partials by term kind
    std::vector<double> hp((size_t)nitems * ncomp);
    HIPCHK(hipMemcpyAsync(hp.data(), part, 8 * hp.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<double> sw(ncomp, 0.0), sx(ncomp, 0.0), ss(ncomp, 0.0);
    for (int64_t i = 0; i < nitems; ++i) {
      std::vector<double>& dst = i >= it_beg[nchunk] ? ss : (items[i].kind == DC_CROSS ? sx : sw);
      for (int q = 0; q < ncomp; ++q) dst[q] += hp[(size_t)i * ncomp + q];
    }
    const char* nm[3] = {"windows", "cross", "support"};
    std::vector<double>* v[3] = {&sw, &sx, &ss};
    for (int k = 0; k < 3; ++k) {
      std::fprintf(stderr, "grad part %s:", nm[k]);
      for (int q = 0; q < ncomp; ++q) std::fprintf(stderr, " %.12e", (*v[k])[q]);
      std::fprintf(stderr, "\n");
    }
  }
  prof::timed(prof::OTHER, 0.0, st, [&] { launch_reduce_partials(part, nitems, ncomp, at<double>(ar, o_gdev), st); });
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(grad_host, at<double>(ar, o_gdev), 8 * ncomp, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  prof::flush();
  for (int q = 0; q < ncomp; ++q)
    if (!std::isfinite(grad_host[q])) throw Err{LMA_E_NOT_PD, "non-finite gradient"};
}

}  // namespace

void grad_impl(lma_state& f, double* grad, int64_t budget, hipStream_t st) {
  if (budget <= 0) budget = (int64_t)16 << 30;
  if (f.mixed()) {
    grad_run<float>(f, grad, budget, st);
  } else if (std::getenv("LMA_GRAD_F32_FROM_F64")) {
    // diagnostic: the float32 gradient pass on float32 roundings of the float64
    // factors (separates the float32 pass's error from the float32 factors')
    int64_t we = 0, ie = 0;
    for (int64_t m = 0; m < f.M; ++m) {
      we += panel_elems(f.Tm[m], (int)f.Ts + 1);
      ie += (int64_t)f.Tm[m] * TB * TB;
    }
    float* buf = nullptr;
    HIPCHK(hipMalloc(&buf, 4 * (we + ie)));
    launch_cast(f.ptr<double>(f.o_win), buf, we, st);
    launch_cast(f.ptr<double>(f.o_win_inv), buf + we, ie, st);
    HIPCHK(hipGetLastError());
    try {
      grad_run<float>(f, grad, budget, st, buf, buf + we, 4 * (we + ie));
    } catch (...) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(buf);
      throw;
    }
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipFree(buf));
  } else {
    grad_run<double>(f, grad, budget, st);
  }
}

}  // namespace lmart
