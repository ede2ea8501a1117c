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
hipError_t engine_init();

}  // namespace lma

namespace lma {

// Per-window geometry used by the vector solves and the mean kernel.
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
};

// Vector solves with the stored window factors:
//   xJ = R_{J_m}^-1 rhsJ,  xW = R_{W_m}^-1 rhsW   (R_W = L11 L11^T, the leading block)
// rhs is gathered from a per-point array (c - K_DS g) or taken per window.
template <typename TW>
struct VecSolveArgs {
  WinTab w;
  const TW* panels;
  const TW* invs;
  const double* rhs_pt;    // per training point, or null
  const double* rhsJ;      // per window layout when rhs_pt is null
  const double* rhsW;
  double* tJ;              // scratch, window layout
  double* tW;
  double* xJ;              // outputs, window layout
  double* xW;
  int accumulate;
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

// c' = c - K_DS g per training point.
struct CgArgs {
  int64_t n;
  int d, s;
  const double* Xs;
  const double* Ss;
  const double* c;
  const double* g;
  double sf2;
  double* out;
};

// mean_u = mu + k_u^T g + sum_{m=q-B..q} (K_{u,J_m} xJ_m - V_u . hJ_m)
//                      - sum_{m=q-B..q-1} (K_{u,W_m} xW_m - V_u . hW_m)
struct MeanArgs {
  WinTab w;
  int64_t n_u;
  int B, d, s, sp;
  const int32_t* ublk;
  const double* Us;
  const double* Ss;
  const double* Xs;
  const double* VtU;
  const double* g;
  const double* xJ;
  const double* xW;
  const double* hJ;
  const double* hW;
  double mu, sf2;
  double* mean;
};

template <typename TW>
void launch_vec_solve(const VecSolveArgs<TW>& a, int M, hipStream_t st);
void launch_h(const HArgs& a, hipStream_t st);
void launch_cg(const CgArgs& a, hipStream_t st);
void launch_mean(const MeanArgs& a, hipStream_t st);

}  // namespace lma
