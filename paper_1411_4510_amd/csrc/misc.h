// Argument blocks and launchers of the small kernels around the engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace lma {

constexpr int MAX_D = 64;
constexpr int MAX_SP = 8192;

struct InvEll {
  double v[MAX_D];
};

struct SummaryArgs {
  const double* partial;  // [groups][ntile][128*128]
  int groups, ntile, Ts, sp, s, d;
  const double* Ss;       // scaled support inputs [s][d]
  double sf2, sn2;
  double* Sdd;            // [sp][sp]
  double* ydd;            // [sp]
  double* qsum;           // [1]
};

struct SolveArgs {
  const double* L;      // tiled lower factor: row tile i at L + 128*128*i(i+1)/2, ld (i+1)*128
  const double* inv;    // inverted diagonal tiles [Ts][128][128]
  const double* A;      // the matrix, full [sp][sp]
  const double* b;      // [sp]
  double* g;            // [sp]
  int sp, iters;
};

struct PredArgs {
  int64_t n_u;
  int sp, s, d;
  double* G;            // [n_u][ldG]: G_u (cols < sp), l_u (col sp); becomes E_u, then L^-1 E_u
  int64_t ldG;
  const double* Us;     // scaled test inputs [n_u][d]
  const double* Ss;     // scaled support inputs [s][d]
  const double* VtU;    // [n_u][sp]
  const double* g;      // [sp]
  double mu, sf2, sn2;
  double* mean;         // [n_u] output
  double* var;          // [n_u] output or null
  double* vn;           // [n_u] |V_u|^2
  const double* xi;     // [n_u]
};

template <typename T>
struct XiArgs {
  int64_t n_u;
  int B;
  const int32_t* ublk;   // test block of each test point
  const int64_t* uptr;   // [M+1]
  const int64_t* Xoff;   // element offset of window m's solved test rows
  const int32_t* Tm;     // column tiles of window m
  const int32_t* twm;    // column tiles of W_m
  const T* Xbuf;
  double* xi;
  int32_t m0, m1;        // only windows m0 <= m < m1 contribute
  int32_t accumulate;    // 1: add to xi, 0: overwrite
};

void launch_scale(const double* X, int64_t n, int d, const InvEll& ie, double* o64, float* o32, hipStream_t st);
void launch_center(const double* y, int64_t n, double mu, double* c64, float* c32, hipStream_t st);
void launch_cast(const double* a, float* b, int64_t n, hipStream_t st);
void launch_zero(double* a, int64_t n, hipStream_t st);
void launch_finalize_summary(const SummaryArgs& a, hipStream_t st);
void launch_global_solve(const SolveArgs& a, hipStream_t st);
void launch_pred_E(const PredArgs& a, hipStream_t st);
void launch_pred_var(const PredArgs& a, hipStream_t st);
template <typename T>
void launch_pred_xi(const XiArgs<T>& a, hipStream_t st);
hipError_t misc_init();
hipError_t vecsolve_init();
hipError_t engine_init();

}  // namespace lma

namespace lma {

// Per-window geometry used by the vector solves.
struct WinTab {
  const int64_t* wstart;   // first training row of W_m
  const int64_t* wlen;     // |W_m|
  const int64_t* dstart;   // first training row of D_m
  const int64_t* dlen;     // |D_m|
  const int32_t* T;        // column tiles of window m
  const int32_t* tw;       // column tiles of W_m
  const int64_t* panel;    // element offset of window m's factor panels
  const int64_t* inv;      // element offset of window m's inverted diagonal tiles
  const int64_t* vec;      // offset of window m's vectors (T*128 doubles)
  const int64_t* rhs;      // element offset of window m's right-hand-side rows (support rows, then the output row)
};

// Vector work on the stored window factors (window layout: T*128 doubles per
// window, W_m rows first).  vJ holds vectors of length |J_m|, vW of |W_m|.
template <typename TW>
struct WinVecArgs {
  WinTab w;
  const TW* panels;        // window factor storage
  const TW* invs;          // inverted diagonal tiles
  int sp, s;
  const double* g;         // [sp] (k_ycp)
  double* vJ;
  double* vW;
};


// Global correction of g (mixed precision): H = sum_m (hJ_m - hW_m),
// rho = L_SS (H - L_SS^T g)  (= y_ddot - Sigma_ddot g with exact window solves).
struct GresArgs {
  const double* L;         // tiled Cholesky factor of Sigma_SS
  const double* hJ;
  const double* hW;
  const double* g;
  double* rho;             // [sp]
  int M, sp;
};

// h = V_X x for X = J_m (hJ) and X = W_m (hW).
struct HArgs {
  WinTab w;
  const double* Vt;        // [n][sp]
  const double* xJ;
  const double* xW;
  double* hJ;              // [M][sp]
  double* hW;
  int sp, M;
};



template <typename TW>
void launch_ycp(const WinVecArgs<TW>& a, int M, int maxT, hipStream_t st);
template <typename TW>
void launch_fwd(const WinVecArgs<TW>& a, int M, int maxT, hipStream_t st);
template <typename TW>
void launch_bwd(const WinVecArgs<TW>& a, int M, hipStream_t st);
void launch_gres(const GresArgs& a, hipStream_t st);
// g += dg and t = L_SS^T dg (one workgroup)
void launch_gupdate(const double* L, const double* dg, double* g, double* t, int sp, hipStream_t st);
// out[i] = Vt[i] . t for every training point (one wave per point)
void launch_vdot(const double* Vt, const double* t, double* out, int64_t n, int sp, hipStream_t st);
// gather a per-point vector into window layout (vJ and vW)
void launch_gather(const WinTab& w, const double* pt, double* vJ, double* vW, int M, int maxT, hipStream_t st);
// vJ += alpha * xJ, vW += alpha * xW over the window layout of length nvec
void launch_axpy2(double* vJ, double* vW, const double* xJ, const double* xW, double alpha, int64_t nvec,
                  hipStream_t st);
void launch_h(const HArgs& a, hipStream_t st);

}  // namespace lma
