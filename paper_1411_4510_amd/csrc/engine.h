// Tiled left-looking Cholesky / triangular-solve engine for gfx950.
//
// A "problem" is a symmetric positive-definite matrix given tile by tile
// (the J rows) plus right-hand-side rows (RHS rows) that are solved against
// its Cholesky factor on the fly: for RHS rows b the engine produces
// b L^-T, i.e. rows of (L^-1 b^T)^T.  Every entry of the matrix and of the
// right-hand sides is generated inside the update kernel (covariance tile,
// explicit matrix, the centred output vector, or a read of the residual band)
// and corrected by
//
//   C_ij = K_ij - V_i V_j^T - sum_{k<j} L_ik L_jk^T
//
// where V rows are the whitened support rows V^T = K_XS L_SS^-T of the
// points of the tile (present only when both tiles carry them).  The V term
// turns the covariance into the residual R = Sigma - Q of the paper.  For the
// overlapping windows of the fit, K_ij - V_i V_j^T (with the noise) is formed
// once per point pair into the residual band and read from there.
//
// All problems of one run advance column by column in lock step: for column
// tile j one update launch covers every row tile i >= j of every problem
// (and every RHS row tile), one launch factors the diagonal tiles and
// inverts them, and one launch applies the inverse to the tiles below.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lma {

constexpr int TB = 128;     // tile edge
constexpr int NT = 256;     // threads per workgroup (4 wave64)
constexpr int DIAG_LD = TB + 1;

// SRC_IDENT: the right-hand-side rows are rows kbeg*TB .. kbeg*TB+127 of the
// identity, so the solve produces the matching rows of L^-T (an explicit
// inverse factor); such a row is zero left of column tile kbeg.
// SRC_BAND: matrix rows whose entries K_pq + noise - V_p.V_q are read from the
// precomputed residual band (StepArgs::band, filled by launch_band): windows
// overlap, so each point pair of the band is formed once instead of once per
// window that holds it.  Row and column tiles are runs of consecutive
// training points starting at pt0.
// SRC_TBAND: right-hand-side rows of test points whose residual cross
// covariances R_ux = K_ux - V_u.V_x with the window's training points are read
// from a precomputed test band (entry (u, x) at band[brow[u] + x]); a test point
// sits in B+1 windows, each of which would otherwise form them again.
enum Src : int32_t { SRC_KERNEL = 0, SRC_EXPLICIT = 1, SRC_CVEC = 2, SRC_IDENT = 3, SRC_BAND = 4, SRC_TBAND = 5 };

template <typename T>
struct RowTile {
  T* panel;          // row r of this row tile at panel + r*ld; column tile k at +(k-kbeg)*TB
  int64_t ld;
  const T* vt;       // whitened support rows of the tile's points (row r at vt + r*vld) or null
  const T* xs;       // length-scaled coordinates of the tile's points ([r][d]) or null
  const double* vt64;  // float64 copies used by the mixed-precision update (V part and
  const double* xs64;  // covariance tile in float64); equal to vt / xs in float64 runs
  const T* cv;       // centred outputs y - mu of the tile's points (column side of SRC_CVEC)
  const T* expl;     // explicit entries: row r, global column c at expl[r*eld + c]
  int64_t eld;
  int32_t nvalid;    // rows that are real points / real entries
  int32_t nstore;    // rows physically stored (loads beyond read 0, stores skipped)
  int32_t src;       // Src
  int32_t is_j;      // 1 for rows of the matrix being factored
  int32_t kbeg;      // first column tile stored (the row is zero to its left); 0 except SRC_IDENT
  int32_t pad_;
  int64_t pt0;       // SRC_BAND / SRC_TBAND: index of the tile's first row point (its own point set)
};

struct ProbDesc {
  int32_t T;            // number of column tiles (J row tiles)
  int32_t R;            // number of RHS row tiles
  int32_t first;        // index of its first RowTile (J tiles, then RHS tiles)
  int32_t ld_from;      // first column tile whose log-diagonal counts toward the log-det
  int64_t invdiag_off;  // element offset of its inverted diagonal tiles [T][TB][TB]
};

struct WorkItem {
  int32_t p;
  int32_t tile;   // local row-tile index: 0..T-1 J tiles, T..T+R-1 RHS tiles
};

template <typename T>
struct StepArgs {
  const RowTile<T>* rt;
  const ProbDesc* pd;
  const WorkItem* items;
  int32_t nitems;
  int32_t j;          // column tile of this step
  int32_t vlen;       // length of the whitened support rows (multiple of 16)
  int32_t d;
  int64_t vld;
  double sf2, sn2;
  T* invdiag;
  double* logdiag;    // [problem][maxT]
  int32_t* status;    // [problem], set to 1 when a pivot is not positive
  int32_t maxT;
  // residual band of the SRC_BAND rows: entry (p, q) with q <= p at band[brow[p] + q]
  // (the other triangle by symmetry); for SRC_TBAND rows the test band, entry
  // (u, x) at band[brow[u] + x]; null when no row of the run uses one
  const T* band;
  const int64_t* brow;
};

// Residual band: for training point p in block a, the entries
//   R_pq = sf2 exp(-|x_p - x_q|^2 / 2) + [p == q] sn2 - V_p . V_q
// for q from the first point of block max(0, a - B) up to p, stored in a
// row-major panel per block (the part of the panel right of p is not read).
// One item is a 128 x 128 tile of such a panel; k_band forms it with the V
// products on the float64 matrix cores and the covariance in float64, and
// rounds once to the storage type.
struct BandItem {
  int64_t p0, q0;   // first row / column training point
  int64_t off;      // element offset of entry (p0, q0) in the band
  int64_t ld;       // panel row stride (elements)
  int32_t nr, nc;   // valid rows / columns
};
template <typename T>
struct BandArgs {
  const BandItem* items;
  int32_t nitems;
  int32_t d;
  int32_t vlen;       // length of the whitened support rows (multiple of 16)
  int32_t noise;      // 1: add sn2 where the row and column index agree (rows and columns are one point set)
  int64_t vld;
  const double* Vt;   // whitened support rows of the column points [.][vld]
  const double* Xs;   // length-scaled coordinates of the column points [.][d]
  const double* Vr;   // the same for the row points (a test band: the test points)
  const double* Xr;
  double sf2, sn2;
  T* band;
};
template <typename T>
void launch_band(const BandArgs<T>& a, hipStream_t st);

// Host-side launchers (engine.hip).
// mixed = true (float storage only): the covariance tile and the V_i V_j^T
// correction are formed in float64 (float64 MFMA), the factor updates as
// float32 MFMA products whose sums are folded into float64 every 144 k; the
// tile is rounded to float32 once, after the cancellation.
template <typename T>
void launch_update(const StepArgs<T>& a, bool mixed, hipStream_t st);
template <typename T>
void launch_diag(const StepArgs<T>& a, const int32_t* plist, int np, hipStream_t st);
template <typename T>
void launch_trsm(const StepArgs<T>& a, hipStream_t st);

// Batched float64-accumulating GEMM over tiles: output tile o computes
//   acc = sum_{t in [tneg, t1)} A_t B_t^T - sum_{t in [t0, tneg)} A_t B_t^T
// over the column range [k0, k1) of each term (A_t, B_t rows contiguous in k;
// the tile is 128 x 128) and writes
//   out = (accumulate ? out : 0) + beta * c + alpha * acc
// on its valid rows / columns (c optional).  Operand rows at or past anr / bnr
// are read from row 0, so an output tile must not store rows >= anr or
// columns >= bnr of any of its terms.
template <typename T>
struct GemmTerm {
  const T* a; int64_t lda; int32_t anr;
  const T* b; int64_t ldb; int32_t bnr;
  int32_t k0, k1;        // column range (multiples of 16)
};
struct GemmOut {
  double* out; int64_t ld;
  const double* c; int64_t ldc;   // addend (scaled by beta) or null
  double alpha, beta;
  int32_t rows, cols;    // valid rows / columns of the output tile
  int32_t accumulate;    // 1: add to the output, 0: overwrite
  int32_t t0, tneg, t1;  // terms [t0, tneg) are subtracted, [tneg, t1) added
};
inline GemmOut gemm_out(double* out, int64_t ld, int rows, int cols, int accumulate, int t0) {
  GemmOut o;
  o.out = out;
  o.ld = ld;
  o.c = nullptr;
  o.ldc = 0;
  o.alpha = 1.0;
  o.beta = 0.0;
  o.rows = rows;
  o.cols = cols;
  o.accumulate = accumulate;
  o.t0 = o.tneg = o.t1 = t0;
  return o;
}
template <typename T>
void launch_tile_gemm(const GemmTerm<T>* terms, const GemmOut* outs, int nout, hipStream_t st);

}  // namespace lma
