// Internal declarations shared by the kernels (kernels.hip) and the host
// driver (api.hip, linalg.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "bmg.h"

namespace bmg {

typedef uint16_t bf16_t;  // BF16 storage: the upper 16 bits of an FP32 (RNE)

// Sets the calling thread's bmg_last_error() message and returns s.
bmg_status set_error(bmg_status s, const std::string &msg);

// One compressed orientation of Omega (rows of A for the CSR orientation,
// rows of A^T for the column-major copy) plus its load-balancing plan:
//   short rows (length <= LONG_ROW entries) are processed one row per lane
//   group, in order of decreasing length so the groups of a wave finish together;
//   long rows are cut into pieces, one wave per piece, whose partial row
//   results are summed in piece order by a fix-up pass.  A piece holds at most
//   LONG_ROW entries and is cut where the row crosses into another column range
//   (ranges of about RANGE_COLS columns of the gathered side) once it holds
//   PIECE_MIN entries.  Pieces are numbered row by row and launched in order of
//   their first column range (piece_ord), and each XCD takes a contiguous run of
//   that order, so the waves resident on an XCD gather from a narrow window of
//   the other factor that its L2 holds.
constexpr int LONG_ROW = 2048;
constexpr int PIECE_MIN = 512;
constexpr int RANGE_COLS = 4096;
constexpr int MAX_RANGES = 256;

struct Plan {
  int64_t nrows = 0, nnz = 0;
  int64_t ncols = 0;               // rows of the gathered operand (columns of Omega here)
  const int64_t *ptr = nullptr;    // [nrows+1]
  const int32_t *idx = nullptr;    // [nnz] column (or row) index of each entry
  const int32_t *short_rows = nullptr;  // (sampled residual only: null = rows 0 .. n_short-1)
  int64_t n_short = 0;
  const int32_t *piece_row = nullptr;  // [n_pieces] row of each piece (row by row)
  const int64_t *piece_beg = nullptr;  // [n_pieces] entry range [beg, end) of each piece
  const int64_t *piece_end = nullptr;
  const int32_t *piece_ord = nullptr;  // [n_pieces] launch order: slot -> piece
  int64_t n_pieces = 0;
  const int32_t *long_rows = nullptr;
  const int32_t *long_p0 = nullptr;  // [n_long+1] first piece of each long row
  int64_t n_long = 0;
};

// Scratch used by one sparse pass: per-wave scalar partials and per-piece
// vector partials.
struct PassScratch {
  double *wsum = nullptr;      // [max_waves * 2]
  void *partial = nullptr;     // [n_pieces * width] (element type of the pass)
  double *result = nullptr;    // [2] final scalar sums
  double *wpart = nullptr;     // [256 * 2] first-stage sums of wsum
  int64_t partial_bytes = 0;   // capacity of partial
  hipEvent_t ev0 = nullptr;    // if set, recorded around the main kernel launch
  hipEvent_t ev1 = nullptr;
};

// ---------------------------------------------------------------- batched passes
// One sparse pass of one problem, for a launch shared by several problems.
// mode 0: fused residual + product (out = R Y + lam X, a = values);
// mode 1: sampled residual (out = R entries or null, a = values or null);
// mode 2: sparse x dense (out = coef S Y + X M, a = S).
template <typename T, typename TG>
struct PassArg {
  Plan pl;
  const T *a = nullptr;
  const T *X = nullptr;
  const TG *Y = nullptr;
  const T *M = nullptr;
  T *out = nullptr;
  T *partial = nullptr;
  double *wsum = nullptr;
  double *result = nullptr;
  int64_t partial_bytes = 0;
  double lam = 0.0, coef = 0.0;
  int ldx = 0, ldy = 0, width = 0, ldo = 0, kx = 0, ldm = 0;
};
constexpr int BATCH_MAX = 8;
template <typename T, typename TG>
struct BatchArg {
  PassArg<T, TG> d[BATCH_MAX];
  int64_t b0[BATCH_MAX + 1];   // first block of each pass (multiples of 8)
  int nd;
};
// Launches nd passes of the same mode and width class in one grid (plus the
// long-row fix-ups and one scalar reduction per pass); the width of every pass
// must be at most max_width<T>().
template <typename T, typename TG>
hipError_t launch_batch(const PassArg<T, TG> *d, int nd, int mode, hipStream_t s);
// lane-group geometry class of a width (passes of one class can share a launch)
template <typename TG>
int width_class(int width);

// ---------------------------------------------------------------- launchers (kernels.hip)
// All return hipError_t of the launch; widths/ld are in elements.

// Fused sampled residual + sparse product (BM gradient of (MF)):
//   r_p = x_row . y_col - a_p ;  Out_row = sum_p r_p y_col + lam * x_row ;  sums[0] = sum r^2
// T: registers, own rows and outputs; TG: the gathered factor rows.
template <typename T, typename TG>
hipError_t launch_grad(const Plan &pl, const T *a, const T *X, int ldx, const TG *Y, int ldy, int k,
                       double lam, T *Out, int ldo, PassScratch sc, int64_t *waves_out,
                       hipStream_t s);

// Sampled product (no sparse output vector): r_p = x_row . y_col - (a ? a_p : 0),
// optionally stored to R[p]; sums[0] = sum r^2, sums[1] = sum r (r + a).
template <typename T, typename TG>
hipError_t launch_sddmm(const Plan &pl, const T *a, const T *X, int ldx, const TG *Y, int ldy, int k,
                        T *R, PassScratch sc, hipStream_t s);

// C = coef * S B + X M on a column slice of width <= 64*VEC:
//   S values in this orientation's order, B (rows indexed by idx), X own-side
//   factor (kx columns, may be null with kx = 0), M (kx x q, row-major ldm).
template <typename T, typename TG>
hipError_t launch_spmm(const Plan &pl, const T *S, const TG *B, int ldb, int q, double coef,
                       const T *X, int ldx, int kx, const T *M, int ldm, T *C, int ldc,
                       PassScratch sc, hipStream_t s);

// ---------------------------------------------------------------- dense-row panel (panel.hip)
// The rows of Omega (short side) dense enough to be kept as a dense panel over
// all n columns, stored column by column: element (i, j) at j * ldi + i.
template <typename T>
struct PanelArg {
  int P = 0;                       // panel rows
  int64_t n = 0;                   // columns
  int ldi = 0;                     // P rounded up to 16 (slots P..ldi-1 are padding)
  const int32_t *rows = nullptr;   // [ldi] row of Omega of each slot (padding repeats rows[0])
  const T *A = nullptr;            // [n x ldi] observed values, NaN where nothing is observed
  T *R = nullptr;                  // [n x ldi] stored residual, 0 where nothing is observed
};
constexpr int PANEL_KSPLIT = 1024;  // column ranges of the rows product (partials added in order)
constexpr int PANEL_KGROUPS = 16;   // first-stage groups of those partials
// r = X_P Y^T - A (use_a) or X_P Y^T where observed, 0 elsewhere; stored in R
// when store; out[0] = sum r^2, out[1] = sum r (X_P Y^T) (fixed order).  bsum:
// 2 doubles per block (at most bsum_cap blocks), tmp: 512 doubles.
template <typename T>
hipError_t launch_panel_resid(const PanelArg<T> &pa, const T *X, int ldx, const T *Y, int ldy, int k,
                              bool use_a, bool store, double *bsum, int64_t bsum_cap, double *tmp,
                              double *out, hipStream_t s);
// Out[rows[i]] = coef (S^T Y)[i] + X[rows[i]] M (kx x q, may be kx = 0) + lam Xl[rows[i]]
// (Xl may be null) with S = A (NaN as 0) when values, else R; part, part2: partials.
template <typename T>
hipError_t launch_panel_rows(const PanelArg<T> &pa, bool values, const T *Y, int ldy, int q, double coef,
                             const T *X, int ldx, int kx, const T *M, int ldm, double lam, const T *Xl,
                             int ldl, T *Out, int ldo, double *part, int64_t part_cap, double *part2,
                             int64_t part2_cap, hipStream_t s);
// Out (n x q) += coef S X_P with X_P the rows rows[] of X; Xt: q x ldi staging.
template <typename T>
hipError_t launch_panel_cols(const PanelArg<T> &pa, bool values, const T *X, int ldx, int q, double coef,
                             T *Out, int ldo, T *Xt, hipStream_t s);
hipError_t launch_panel_fill(int P, int64_t n, int ldi, const int32_t *rows, const int64_t *ptr,
                             const int32_t *idx, const double *val, double *A, float *A32, hipStream_t s);
hipError_t launch_panel_keep(int64_t nnz, const int32_t *idx, const uint8_t *mask, int32_t *keep,
                             hipStream_t s);
hipError_t launch_panel_compact(int64_t ncols, int64_t nnz, const int64_t *ptr, const int32_t *keep,
                                const int32_t *pos, const int32_t *idx, const double *val, int32_t *ridx,
                                double *rval, int64_t *rptr, hipStream_t s);

// Dense helpers.
template <typename T>
hipError_t launch_gram(int64_t N, int a, const T *X, int ldx, int b, const T *Y, int ldy,
                       double *part, int64_t part_cap, double *out, hipStream_t s);
template <typename T>
hipError_t launch_gemm_ts(int64_t N, int a, const T *X, int ldx, int b, const double *M, int ldm,
                          T *C, int ldc, double beta, hipStream_t s);
template <typename T>
hipError_t launch_fill(T *p, int64_t rows, int cols, int ld, double v, hipStream_t s);
template <typename T>
hipError_t launch_axpy(int64_t rows, int cols, double a, const T *X, int ldx, T *Y, int ldy,
                       hipStream_t s);  // Y += a X
template <typename T>
hipError_t launch_copy_cols(int64_t rows, int cols, const T *X, int ldx, T *Y, int ldy,
                            hipStream_t s);
template <typename Tin, typename Tout>
hipError_t launch_convert(int64_t n, const Tin *x, Tout *y, hipStream_t s);
template <typename Tin, typename Tout>
hipError_t launch_convert_cols(int64_t rows, int cols, const Tin *X, int ldx, Tout *Y, int ldy,
                               hipStream_t s);
template <typename T>
hipError_t launch_normals(uint64_t seed, uint64_t stream, int64_t rows, int cols, int ld, T *out,
                          hipStream_t s);  // entry (i, j) is normal number i*cols + j
hipError_t launch_gather_perm(int64_t nnz, const int32_t *perm, const double *in, double *out,
                              hipStream_t s);
hipError_t launch_reduce_wsum(const double *wsum, int64_t waves, int nsum, double *tmp, double *out,
                              hipStream_t s);
// Setup helpers.
hipError_t launch_row_ids(int64_t m, const int64_t *row_ptr, int32_t *rid, hipStream_t s);
hipError_t launch_iota(int64_t n, int32_t *p, hipStream_t s);
hipError_t launch_gather_csc(int64_t nnz, const int32_t *perm, const int32_t *rid,
                             const double *val, int32_t *crow, double *cval, hipStream_t s);
hipError_t launch_col_ptr(int64_t nnz, int64_t n, const int32_t *sorted_col, int64_t *cptr,
                          hipStream_t s);
hipError_t launch_range_bounds(const int64_t *ptr, const int32_t *idx, const int32_t *rows,
                               int64_t n, int nr, int64_t wc, int32_t *out, hipStream_t s);
hipError_t launch_check_csr(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
                            const double *val, const int32_t *rid, int *flags, hipStream_t s);

// polyMF-SS column passes (colpass.hip).  Per block j every row of each side
// has a record {prev, step, x, dir}: the value of block j-1 after its step,
// that step, the value of block j, and block j's direction.
template <typename T>
struct alignas(4 * sizeof(T)) Q4 {
  T x, y, z, w;
};
// records of block 0: {0, 0, W[i, 0], 0} and {0, 0, H[l, 0], 0}
template <typename T>
hipError_t launch_col_pack0(int64_t m, int64_t n, const T *W, const T *H, int ld, Q4<T> *Gm, Q4<T> *Gn,
                            hipStream_t s);
// One orientation (own records Gown, gathered records Goth): with upd, the
// stored residual takes the previous block's step,
//   r += s_row y'_l + x'_row s_l - s_row s_l;
// then Gown[row].w = -(sum r y_l + lam x_row) / (sum y_l^2 + lam).
// part: 2 doubles per piece of the plan.
template <typename T>
hipError_t launch_col_grad(const Plan &pl, T *r, Q4<T> *Gown, const Q4<T> *Goth, bool upd, double lam,
                           double *part, hipStream_t s);
// out[0..4] = sum over Omega (rows orientation) of r a, a^2, r b, a b, b^2 with
// a = dw_i h_l + w_i dh_l, b = dw_i dh_l; out[5..8] = w.dw, dw.dw, h.dh, dh.dh.
// bpart: 5 doubles per 4 work units (bpart_cap doubles); dpart: 512 doubles.
// With state (device, or null), also the block's step from those sums: the
// quartic c1 = h0 + lam (h5 + h7), c2 = h1 / 2 + h2 + lam (h6 + h8) / 2,
// c3 = h3, c4 = h4 / 2 and t = quartic_min(c1..c4) into state[0]; state[1]
// counts the blocks with t > 0, state[2] is set to 1 (and t to 0) when a
// coefficient is not finite.
template <typename T>
hipError_t launch_col_quartic(const Plan &pl, const T *r, int64_t m, int64_t n, const Q4<T> *Gm,
                              const Q4<T> *Gn, double *bpart, int64_t bpart_cap, double *dpart,
                              double *out, double lam, double *state, hipStream_t s);
// Block j moves by t = *tp (device) along its direction: X[:, j] += t dir;
// the records are rewritten for block jn (jn < 0: none).
template <typename T>
hipError_t launch_col_step(int64_t m, int64_t n, T *W, T *H, int ld, int j, int jn, const double *tp,
                           Q4<T> *Gm, Q4<T> *Gn, hipStream_t s);

// Kernel-estimation QSDP pair passes (rke.hip), FP64, rows plan of a
// symmetric Omega, factor W (n x k, ld):
//   r_p = ||w_i - w_j||^2 - d2_p (stored), deg_i = sum r, adeg_i = sum |r|,
//   out[0] = sum r^2; part: 2 doubles per piece; bpart: 1 double per 4 units.
hipError_t launch_rke_res(const Plan &pl, const double *W, int ld, int k, const double *d2, double *r,
                          double *deg, double *adeg, double *part, double *bpart, int64_t bpart_cap,
                          double *out, hipStream_t s);
// out[0..4] = sum of r a1, a1^2, r a2, a1 a2, a2^2 with a1 = (w_i - w_j).(d_i - d_j),
// a2 = ||d_i - d_j||^2 (D at the same ld); bpart: 5 doubles per 4 units.
hipError_t launch_rke_quartic(const Plan &pl, const double *W, const double *D, int ld, int k,
                              const double *r, double *bpart, int64_t bpart_cap, double *out,
                              hipStream_t s);
// out[j] = <A[j], B[j]> (Frobenius) for j < np <= 4, n x k at ld; bpart: 512 doubles
hipError_t launch_frob_dots(int64_t n, int k, int ld, const double *const *A, const double *const *B, int np,
                            double *bpart, double *out, hipStream_t s);
// Out = deg U - Out (row scaling)
hipError_t launch_rowscale_sub(int64_t n, int q, const double *deg, const double *U, int ldu, double *Out,
                               int ldo, hipStream_t s);
// V = J V: subtract each column's mean (part: 64 q doubles of scratch)
hipError_t launch_center_cols(int64_t n, int q, double *V, int ld, double *part, int64_t part_cap,
                              hipStream_t s);
// flag[0] = 1 where the two orientations' indices or values differ
hipError_t launch_cmp_orient(int64_t nnz, const int32_t *a, const int32_t *b, const double *va,
                             const double *vb, int *flag, hipStream_t s);

// Widest slice one launch handles for element type T.
// (8 lanes x 16 bytes per chunk, at most 8 chunks: 128 doubles / 256 floats)
template <typename T> constexpr int max_width() { return 128 * (16 / (int)sizeof(T)); }


// Global minimiser over t >= 0 of psi(t) = c1 t + c2 t^2 + c3 t^3 + c4 t^4
// (c4 >= 0): psi' is a cubic; the real roots of psi'' cut [0, B] (B a bound on
// the roots of psi') into intervals where psi' is monotone, safeguarded
// Newton (bisection every second step) finds the root in each interval where
// psi' changes sign, and the best of t = 0 and those roots is returned.  The
// same code runs on the host and on the device (no contraction into fused
// multiply-adds, so both give the same t).
__host__ __device__ inline double quartic_min(double c1, double c2, double c3, double c4) {
#pragma clang fp contract(off)
  const double a = 4.0 * c4, b = 3.0 * c3, c = 2.0 * c2, d = c1;
  double B;
  if (a > 0.0) B = 1.0 + fmax(fmax(fabs(b), fabs(c)), fabs(d)) / a;
  else if (b != 0.0) B = 1.0 + fmax(fabs(c), fabs(d)) / fabs(b);
  else if (c != 0.0) B = 1.0 + fabs(d / c);
  else return 0.0;
  double cut[4];
  int nc = 0;
  cut[nc++] = 0.0;
  // roots of psi'' = c + 2 b t + 3 a t^2
  if (a > 0.0) {
    const double disc = 4.0 * b * b - 12.0 * a * c;
    if (disc > 0.0) {
      const double sq = sqrt(disc);
      const double q = -0.5 * (2.0 * b + (b >= 0.0 ? sq : -sq));
      double r1 = q / (3.0 * a), r2 = q != 0.0 ? c / q : r1;
      if (r1 > r2) { const double tmp = r1; r1 = r2; r2 = tmp; }
      if (r1 > 0.0 && r1 < B) cut[nc++] = r1;
      if (r2 > 0.0 && r2 < B && r2 != r1) cut[nc++] = r2;
    }
  } else if (b != 0.0) {
    const double r = -c / (2.0 * b);
    if (r > 0.0 && r < B) cut[nc++] = r;
  }
  cut[nc++] = B;
  double best = 0.0, fbest = 0.0;
  for (int i = 0; i + 1 < nc; ++i) {
    double lo = cut[i], hi = cut[i + 1];
    double flo = ((a * lo + b) * lo + c) * lo + d, fhi = ((a * hi + b) * hi + c) * hi + d;
    if (flo == 0.0) { hi = lo; fhi = 0.0; }
    else if ((flo < 0.0) == (fhi < 0.0) && fhi != 0.0) continue;
    // safeguarded Newton on psi' inside the bracket: a Newton step from the
    // end with the smaller |psi'| when it lands strictly inside, else the
    // midpoint; every second step bisects, so the bracket at least halves
    // every two steps; stop once a Newton step moves by at most a few ulps
    // or the bracket cannot shrink
    for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
      double x = 0.5 * (lo + hi);
      bool conv = false;
      if (!(it & 1)) {
        const bool lside = fabs(flo) < fabs(fhi);
        const double x0 = lside ? lo : hi, f0 = lside ? flo : fhi;
        const double d0 = (3.0 * a * x0 + 2.0 * b) * x0 + c;
        if (d0 != 0.0) {
          const double xn = x0 - f0 / d0;
          if (xn > lo && xn < hi) {
            x = xn;
            conv = fabs(xn - x0) <= 4.0 * 2.220446049250313e-16 * fabs(x0);
          }
        }
      }
      if (x <= lo || x >= hi) break;
      const double fm = ((a * x + b) * x + c) * x + d;
      if ((fm < 0.0) == (flo < 0.0) && fm != 0.0) { lo = x; flo = fm; }
      else { hi = x; fhi = fm; }
      if (fm == 0.0 || conv) break;
    }
    const double t = fabs(flo) < fabs(fhi) ? lo : hi;
    const double ft = (((c4 * t + c3) * t + c2) * t + c1) * t;
    if (t > 0.0 && ft < fbest) { best = t; fbest = ft; }
  }
  return best;
}

}  // namespace bmg

#include "linalg.h"
