// Dense-row panel of the sparse passes (gfx950).
//
// Rows of Omega (on the short side) at least as dense as a threshold are
// taken out of the gather path and kept as a dense panel over all n columns:
// the observed values A_P with NaN where nothing is observed, and the stored
// residual R_P with zeros there.  Every product with those rows is then a
// dense contraction that streams the panel and the n-side operand once, on the
// FP64 matrix cores (16x16x4 FP64 MFMA, operands converted to FP64 in
// registers), instead of gathering one factor row per stored entry.  The panel
// is stored column by column (element (i, j) at j * ldi + i, ldi = P rounded up
// to 16; rows P..ldi-1 are padding: unobserved, and their row index repeats a
// real one), so that a block working on a range of columns streams one
// contiguous stretch of it.  Three kernels cover every pass:
//   k_panel_resid: D = Y X_P^T (n x P), r = D - A (or D) where observed, 0 else;
//                  optional store of r into R_P, block sums of r^2 and r D;
//   k_panel_rows:  Out_P = coef S^T Y (+ X_P M + lam X_P) with S = R_P or A_P,
//                  split over column ranges with partials added in order;
//   k_panel_cols:  Out += coef S X_P (every output element owned by one lane),
//                  X_P first transposed into a small staging block.
// MFMA layouts (FP64 16x16x4): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; register v of lane l holds D[4 v + l / 16][l % 16].  The
// contraction index is taken 16 at a time: in MFMA step s lane (kr, cl) = (l / 16,
// l % 16) supplies index f0 + 4 kr + s, so that a lane's four values of one row
// are adjacent.  All sums are taken in a fixed order: results are bitwise
// reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <mutex>

#include "bmg_internal.h"

namespace bmg {

typedef double d4p_t __attribute__((ext_vector_type(4)));

// Four consecutive elements p[0..3] (those at or beyond lim read as 0) as FP64.
template <typename T>
__device__ __forceinline__ void ld4(const T *__restrict__ p, int f0, int lim, double (&x)[4]) {
  if (f0 + 4 <= lim) {
    if constexpr (sizeof(T) == 8) {
      const double2 a = *reinterpret_cast<const double2 *>(p + f0);
      const double2 b = *reinterpret_cast<const double2 *>(p + f0 + 2);
      x[0] = a.x; x[1] = a.y; x[2] = b.x; x[3] = b.y;
    } else {
      const float4 a = *reinterpret_cast<const float4 *>(p + f0);
      x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    }
    return;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) x[e] = (f0 + e < lim) ? (double)p[f0 + e] : 0.0;
}

// ------------------------------------------------------------------ residual
// Block bx: column tile bx (16 columns); wave w: panel-row tiles w, w + 4,
// w + 8, w + 12.  M = columns j, N = panel rows i, K = k (16 at a time, then
// the last k % 16 four at a time).
template <typename T>
__global__ __launch_bounds__(256) void k_panel_resid(int TI, int64_t n, int k,
                                                     const int32_t *__restrict__ rows,
                                                     const T *__restrict__ X, int ldx,
                                                     const T *__restrict__ Y, int ldy,
                                                     const T *__restrict__ A, int ldi, int use_a,
                                                     T *__restrict__ R, double *__restrict__ bsum) {
  __shared__ double red[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kr = lane / 16, cl = lane % 16;
  const int64_t j0 = (int64_t)blockIdx.x * 16;
  d4p_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = d4p_t{0.0, 0.0, 0.0, 0.0};
  const int64_t ja = j0 + cl;
  const bool jv = ja < n;
  const T *yrow = Y + (jv ? ja : 0) * ldy;
  const T *xrow[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int it = wave + 4 * t;
    xrow[t] = X + (int64_t)rows[(it < TI ? it : 0) * 16 + cl] * ldx;
  }
  const int k16 = k / 16 * 16;
  for (int f0 = 0; f0 < k16; f0 += 16) {
    const int fl = f0 + 4 * kr;
    double a[4];
    ld4(yrow, fl, jv ? k : 0, a);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (wave + 4 * t >= TI) break;
      double b[4];
      ld4(xrow[t], fl, k, b);
#pragma unroll
      for (int st = 0; st < 4; ++st) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b[st], acc[t], 0, 0, 0);
    }
  }
  for (int f0 = k16; f0 < k; f0 += 4) {
    const int f = f0 + kr;
    const double a = (jv && f < k) ? (double)yrow[f] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (wave + 4 * t >= TI) break;
      const double b = f < k ? (double)xrow[t][f] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
  double ss = 0.0, sx = 0.0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int it = wave + 4 * t;
    if (it >= TI) break;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t j = j0 + 4 * v + kr;
      if (j < n) {
        const int64_t off = j * ldi + it * 16 + cl;
        const double av = (double)A[off];
        const double d = acc[t][v];
        const bool obs = !isnan(av);
        const double r = obs ? (use_a ? d - av : d) : 0.0;
        const T rt = (T)r;
        if (R) R[off] = rt;
        // sums of what the stored (rounded) residual holds, as the sparse passes do
        const double rr = (double)rt;
        ss += rr * rr;
        sx += rr * d;
      }
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    ss += __shfl_xor(ss, o, 64);
    sx += __shfl_xor(sx, o, 64);
  }
  if (lane == 0) {
    red[0][wave] = ss;
    red[1][wave] = sx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bsum[2 * blockIdx.x] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    bsum[2 * blockIdx.x + 1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  }
}

template <typename T>
hipError_t launch_panel_resid(const PanelArg<T> &pa, const T *X, int ldx, const T *Y, int ldy, int k,
                              bool use_a, bool store, double *bsum, int64_t bsum_cap, double *tmp,
                              double *out, hipStream_t s) {
  if (pa.P <= 0 || (ldx % 4) || (ldy % 4) || (pa.ldi % 16)) return hipErrorInvalidValue;
  const int TI = pa.ldi / 16;
  if (TI > 16) return hipErrorInvalidValue;
  const int64_t nb = (pa.n + 15) / 16;
  if (nb > bsum_cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_panel_resid<T>), dim3((unsigned)nb), dim3(256), 0, s, TI, pa.n, k, pa.rows, X, ldx, Y,
                     ldy, pa.A, pa.ldi, use_a ? 1 : 0, store ? pa.R : (T *)nullptr, bsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_wsum(bsum, nb, 2, tmp, out, s);
}

// X_P^T: Xt[c][s] = X[rows[s]][c] for the ldi panel slots s and c < q (ld ldi)
template <typename T>
__global__ void k_panel_xt(int ldi, int q, const int32_t *__restrict__ rows, const T *__restrict__ X, int ldx,
                           T *__restrict__ Xt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ldi * q) return;
  const int c = e / ldi, sl = e % ldi;
  Xt[(int64_t)c * ldi + sl] = X[(int64_t)rows[sl] * ldx + c];
}

// ------------------------------------------------------------------ rows product
// Block (bx, by): columns [bx cpb, (bx + 1) cpb) (cpb a multiple of 16); wave w:
// panel-row tiles 4 NT by + w + 4 t (t < NT) and every output column tile (NQ =
// ceil(q / 16) of them).  The NT tiles of a wave share every loaded Y value, and
// one block reads each Y row once for all the panel rows it covers; operands are
// loaded at the start of each 16-column step (no second register set: the
// registers go to the NT x NQ accumulators).  M = panel rows i, N = output
// columns c, K = columns j.  part[bx][i][c] (ldi x 16 NQ per block) gets the
// block's partial sums.
template <typename T, int NQ, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NQ * NT >= 9 ? 3 : 1))) void k_panel_rows(int TI, int64_t n, int q, int64_t cpb,
                                                    const T *__restrict__ S, int ldi, int values,
                                                    const T *__restrict__ Y, int ldy,
                                                    double *__restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kr = lane / 16, cl = lane % 16;
  const int Q16 = NQ * 16;
  const int tb = blockIdx.y * 4 * NT + wave;
  if (tb >= TI) return;   // whole wave
  const int64_t c0 = (int64_t)blockIdx.x * cpb;
  const int64_t c1 = (c0 + cpb) < n ? (c0 + cpb) : n;
  int ir[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int ti = tb + 4 * t;
    ir[t] = (ti < TI ? ti : tb) * 16 + cl;
  }
  d4p_t acc[NT][NQ];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int u = 0; u < NQ; ++u) acc[t][u] = d4p_t{0.0, 0.0, 0.0, 0.0};
  for (int64_t jj = c0; jj < c1; jj += 16) {
    double a[NT][4], b[4][NQ];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int64_t j = jj + 4 * kr + st;
      const bool jv = j < c1;
      const int64_t jc = jv ? j : c0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        double x = (double)S[jc * ldi + ir[t]];
        if (values) x = isnan(x) ? 0.0 : x;
        a[t][st] = jv ? x : 0.0;
      }
      const T *yr = Y + jc * ldy;
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        const int c = u * 16 + cl;
        b[st][u] = (jv && c < q) ? (double)yr[c] : 0.0;
      }
    }
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int u = 0; u < NQ; ++u)
          acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t][st], b[st][u], acc[t][u], 0, 0, 0);
  }
  double *pb = part + (int64_t)blockIdx.x * TI * 16 * Q16;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int ti = tb + 4 * t;
    if (ti >= TI) break;
#pragma unroll
    for (int u = 0; u < NQ; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ii = ti * 16 + 4 * v + kr, c = u * 16 + cl;
        pb[(int64_t)ii * Q16 + c] = acc[t][u][v];
      }
  }
}

// Stage 1 of the partial sums: part2[g][i][c] = sum over blocks b of group g
// (b = g bpg .. g bpg + bpg - 1, in order) of part[b][i][c].
__global__ __launch_bounds__(256) void k_panel_rows_sum(int P16, int Q16, int nbk, int bpg,
                                                        const double *__restrict__ part,
                                                        double *__restrict__ part2) {
  const int64_t E = (int64_t)P16 * Q16;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int g = blockIdx.y;
  const int b0 = g * bpg, b1 = (b0 + bpg) < nbk ? (b0 + bpg) : nbk;
  double s = 0.0;
  for (int b = b0; b < b1; ++b) s += part[(int64_t)b * E + e];
  part2[(int64_t)g * E + e] = s;
}

// Out[rows[i]][c] = coef * sum_g part2[g][i][c] (groups in order)
//                   + sum_{r < kx} X[rows[i]][r] M[r][c] + lam Xl[rows[i]][c]
template <typename T>
__global__ __launch_bounds__(256) void k_panel_rows_fix(int P, int q, int P16, int Q16, int ng,
                                                        const double *__restrict__ part2,
                                                        const int32_t *__restrict__ rows, double coef,
                                                        const T *__restrict__ X, int ldx, int kx,
                                                        const T *__restrict__ M, int ldm, double lam,
                                                        const T *__restrict__ Xl, int ldl,
                                                        T *__restrict__ Out, int ldo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)P * q) return;
  const int i = (int)(e / q), c = (int)(e % q);
  const int64_t E = (int64_t)P16 * Q16;
  double sum = 0.0;
  for (int g = 0; g < ng; ++g) sum += part2[(int64_t)g * E + (int64_t)i * Q16 + c];
  const int64_t row = rows[i];
  double v = coef * sum;
  for (int r = 0; r < kx; ++r) v += (double)X[row * ldx + r] * (double)M[(int64_t)r * ldm + c];
  if (Xl) v += lam * (double)Xl[row * ldl + c];
  Out[row * ldo + c] = (T)v;
}

template <typename T>
hipError_t launch_panel_rows(const PanelArg<T> &pa, bool values, const T *Y, int ldy, int q, double coef,
                             const T *X, int ldx, int kx, const T *M, int ldm, double lam, const T *Xl,
                             int ldl, T *Out, int ldo, double *part, int64_t part_cap, double *part2,
                             int64_t part2_cap, hipStream_t s) {
  if (pa.P <= 0 || q <= 0 || (pa.ldi % 16)) return hipErrorInvalidValue;
  const int TI = pa.ldi / 16, TQ = (q + 15) / 16;
  if (TQ > 12) return hipErrorInvalidValue;
  const int P16 = pa.ldi, Q16 = TQ * 16;
  const int64_t per = (int64_t)P16 * Q16;
  int64_t nbk = PANEL_KSPLIT;
  if (nbk * per > part_cap) nbk = part_cap / per;
  if (nbk < 1) return hipErrorInvalidValue;
  int64_t cpb = (pa.n + nbk - 1) / nbk;
  cpb = (cpb + 15) / 16 * 16;
  nbk = (pa.n + cpb - 1) / cpb;
  int ng = (int)std::min<int64_t>(PANEL_KGROUPS, nbk);
  if ((int64_t)ng * per > part2_cap) return hipErrorInvalidValue;
  const int bpg = (int)((nbk + ng - 1) / ng);
  ng = (int)((nbk + bpg - 1) / bpg);
  // panel-row tiles per wave: as many as the accumulators allow (NT NQ <= 12)
  const int ntc = TQ <= 3 ? 4 : (TQ == 4 ? 3 : (TQ <= 6 ? 2 : 1));
  const int NTr = std::min((TI + 3) / 4, ntc);
  const dim3 grid((unsigned)nbk, (unsigned)((TI + 4 * NTr - 1) / (4 * NTr)));
  const T *Sp = values ? pa.A : (const T *)pa.R;
#define BMG_PANEL_ROWS(NQv, NTv)                                                                            \
  hipLaunchKernelGGL((k_panel_rows<T, NQv, NTv>), grid, dim3(256), 0, s, TI, pa.n, q, cpb, Sp, pa.ldi,      \
                     values ? 1 : 0, Y, ldy, part)
#define BMG_PANEL_ROWS_NT(NQv, NTMAX)                                                                       \
  do {                                                                                                      \
    if (NTr >= 4 && NTMAX >= 4) BMG_PANEL_ROWS(NQv, (NTMAX >= 4 ? 4 : 1));                                 \
    else if (NTr == 3 && NTMAX >= 3) BMG_PANEL_ROWS(NQv, (NTMAX >= 3 ? 3 : 1));                            \
    else if (NTr == 2 && NTMAX >= 2) BMG_PANEL_ROWS(NQv, (NTMAX >= 2 ? 2 : 1));                            \
    else BMG_PANEL_ROWS(NQv, 1);                                                                            \
  } while (0)
  switch (TQ) {
    case 1: BMG_PANEL_ROWS_NT(1, 4); break;
    case 2: BMG_PANEL_ROWS_NT(2, 4); break;
    case 3: BMG_PANEL_ROWS_NT(3, 4); break;
    case 4: BMG_PANEL_ROWS_NT(4, 3); break;
    case 5: BMG_PANEL_ROWS_NT(5, 2); break;
    case 6: BMG_PANEL_ROWS_NT(6, 2); break;
    case 7: BMG_PANEL_ROWS(7, 1); break;
    case 8: BMG_PANEL_ROWS(8, 1); break;
    case 9: BMG_PANEL_ROWS(9, 1); break;
    case 10: BMG_PANEL_ROWS(10, 1); break;
    case 11: BMG_PANEL_ROWS(11, 1); break;
    default: BMG_PANEL_ROWS(12, 1); break;
  }
#undef BMG_PANEL_ROWS_NT
#undef BMG_PANEL_ROWS
  hipLaunchKernelGGL(k_panel_rows_sum, dim3((unsigned)((per + 255) / 256), (unsigned)ng), dim3(256), 0, s, P16,
                     Q16, (int)nbk, bpg, (const double *)part, part2);
  const int64_t el = (int64_t)pa.P * q;
  hipLaunchKernelGGL((k_panel_rows_fix<T>), dim3((unsigned)((el + 255) / 256)), dim3(256), 0, s, pa.P, q, P16,
                     Q16, ng, (const double *)part2, pa.rows, coef, X, ldx, kx, M, ldm, lam, Xl, ldl, Out, ldo);
  return hipGetLastError();
}

// ------------------------------------------------------------------ columns product
// Block bx: columns [64 bx, +64), wave w: column tile 4 bx + w and every
// output column tile (at most NQ).  M = columns j, N = output columns c,
// K = panel rows i; X_P comes transposed (Xt, ld ldi) so that a lane's four
// values of one output column are adjacent.
template <typename T, int NQ>
__global__ __launch_bounds__(256) void k_panel_cols(int TI, int64_t n, int q, const T *__restrict__ S, int ldi,
                                                    int values, const T *__restrict__ Xt, double coef,
                                                    T *__restrict__ Out, int ldo) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kr = lane / 16, cl = lane % 16;
  const int64_t j0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int TQ = (q + 15) / 16;
  d4p_t acc[NQ];
#pragma unroll
  for (int u = 0; u < NQ; ++u) acc[u] = d4p_t{0.0, 0.0, 0.0, 0.0};
  const int64_t ja = j0 + cl;
  const bool jv = ja < n;
  const T *srow = S + (jv ? ja : 0) * ldi;
  // the panel values of the next 16 rows are loaded before the products of
  // the current ones are issued
  double an[4];
  ld4(srow, 4 * kr, jv ? ldi : 0, an);
  for (int ii = 0; ii < TI * 16; ii += 16) {
    double a[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) a[e] = an[e];
    if (ii + 16 < TI * 16) ld4(srow, ii + 16 + 4 * kr, jv ? ldi : 0, an);
    if (values) {
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = isnan(a[e]) ? 0.0 : a[e];
    }
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      if (u >= TQ) break;
      const int c = u * 16 + cl;
      double b[4];
      ld4(Xt + (int64_t)(c < q ? c : 0) * ldi, ii + 4 * kr, c < q ? ldi : 0, b);
#pragma unroll
      for (int st = 0; st < 4; ++st) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b[st], acc[u], 0, 0, 0);
    }
  }
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    if (u >= TQ) break;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t j = j0 + 4 * v + kr;
      const int c = u * 16 + cl;
      if (j < n && c < q) {
        const int64_t o = j * ldo + c;
        Out[o] = (T)((double)Out[o] + coef * acc[u][v]);
      }
    }
  }
}

// Same product as k_panel_cols (the same MFMA sequence, so the same bits), with
// X_P held in LDS: each block first gathers the q columns of the panel rows of
// X there as FP64, row c of the copy at c (ldi + 2) (the two-element pad puts
// the 16 lanes of a fragment read on distinct banks), then its waves take
// column tiles 4 b + w, 4 (b + G) + w, ... (G blocks, as many as are resident
// on the device at once).  Per tile the output rows are loaded at the start and
// the panel values of four K steps one group ahead.
template <typename T, int NQ>
__global__ __launch_bounds__(256) void k_panel_cols_lds(int TI, int64_t n, int q, const T *__restrict__ S,
                                                        int ldi, int values, const int32_t *__restrict__ rows,
                                                        const T *__restrict__ X, int ldx, double coef,
                                                        T *__restrict__ Out, int ldo) {
  extern __shared__ double xs[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kr = lane / 16, cl = lane % 16;
  const int ls = ldi + 2;
  for (int e = threadIdx.x; e < q * ldi; e += 256) {
    const int i = e / q, c = e % q;
    xs[c * ls + i] = (double)X[(int64_t)rows[i] * ldx + c];
  }
  __syncthreads();
  const int64_t tiles = (n + 15) / 16;
  for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < tiles; t += (int64_t)gridDim.x * 4) {
    const int64_t j0 = t * 16;
    d4p_t acc[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) acc[u] = d4p_t{0.0, 0.0, 0.0, 0.0};
    const int64_t ja = j0 + cl;
    const bool jv = ja < n;
    const T *srow = S + (jv ? ja : 0) * ldi;
    double ov[NQ][4];
#pragma unroll
    for (int u = 0; u < NQ; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = j0 + 4 * v + kr;
        const int c = u * 16 + cl;
        ov[u][v] = (j < n && c < q) ? (double)Out[j * ldo + c] : 0.0;
      }
    double nx[4][4];
#pragma unroll
    for (int st = 0; st < 4; ++st) ld4(srow, st * 16 + 4 * kr, (jv && st < TI) ? ldi : 0, nx[st]);
    for (int g = 0; g < TI; g += 4) {
      double cu[4][4];
#pragma unroll
      for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int e = 0; e < 4; ++e) cu[st][e] = nx[st][e];
      if (g + 4 < TI) {
#pragma unroll
        for (int st = 0; st < 4; ++st)
          ld4(srow, (g + 4 + st) * 16 + 4 * kr, (jv && g + 4 + st < TI) ? ldi : 0, nx[st]);
      }
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        if (g + h >= TI) break;
        const int ii = (g + h) * 16;
        double a[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = (values && isnan(cu[h][e])) ? 0.0 : cu[h][e];
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
          const int c = u * 16 + cl;
          double b[4];
          if (c < q) {
            const double2 b0 = *reinterpret_cast<const double2 *>(xs + c * ls + ii + 4 * kr);
            const double2 b1 = *reinterpret_cast<const double2 *>(xs + c * ls + ii + 4 * kr + 2);
            b[0] = b0.x; b[1] = b0.y; b[2] = b1.x; b[3] = b1.y;
          } else {
            b[0] = b[1] = b[2] = b[3] = 0.0;
          }
#pragma unroll
          for (int st = 0; st < 4; ++st)
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b[st], acc[u], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < NQ; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = j0 + 4 * v + kr;
        const int c = u * 16 + cl;
        if (j < n && c < q) Out[j * ldo + c] = (T)(ov[u][v] + coef * acc[u][v]);
      }
  }
}

// Blocks of 256 threads of kernel fn with lds bytes of dynamic LDS that are
// resident on the current device at once (0: none fit); cached per device,
// kernel and size.
static int64_t resident_blocks(const void *fn, size_t lds) {
  struct Ent {
    int dev;
    const void *fn;
    size_t lds;
    int64_t blocks;
  };
  static std::mutex mu;
  static Ent cache[64];
  static int used = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  {
    std::lock_guard<std::mutex> g(mu);
    for (int e = 0; e < used; ++e)
      if (cache[e].dev == dev && cache[e].fn == fn && cache[e].lds == lds) return cache[e].blocks;
  }
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds) != hipSuccess) {
    (void)hipGetLastError();
    per_cu = 0;
  }
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    cus = 0;
  }
  const int64_t blocks = (int64_t)std::max(per_cu, 0) * std::max(cus, 0);
  std::lock_guard<std::mutex> g(mu);
  if (used < 64) cache[used++] = Ent{dev, fn, lds, blocks};
  return blocks;
}

template <typename T>
hipError_t launch_panel_cols(const PanelArg<T> &pa, bool values, const T *X, int ldx, int q, double coef,
                             T *Out, int ldo, T *Xt, hipStream_t s) {
  if (pa.P <= 0 || q <= 0 || (pa.ldi % 16)) return hipErrorInvalidValue;
  const int TI = pa.ldi / 16, TQ = (q + 15) / 16;
  if (TQ > 12) return hipErrorInvalidValue;
  const T *Sp = values ? pa.A : (const T *)pa.R;
  // X_P in LDS when it fits (at most 5 output column tiles: at 6 the registers
  // leave one wave per SIMD)
  const size_t lds = (size_t)q * (pa.ldi + 2) * sizeof(double);
  if (TQ <= 5 && lds <= 160 * 1024) {
    const void *fn = nullptr;
    switch (TQ) {
      case 1: fn = (const void *)k_panel_cols_lds<T, 1>; break;
      case 2: fn = (const void *)k_panel_cols_lds<T, 2>; break;
      case 3: fn = (const void *)k_panel_cols_lds<T, 3>; break;
      case 4: fn = (const void *)k_panel_cols_lds<T, 4>; break;
      default: fn = (const void *)k_panel_cols_lds<T, 5>; break;
    }
    const int64_t tiles = (pa.n + 15) / 16;
    int64_t nb = std::min(resident_blocks(fn, lds), (tiles + 3) / 4);
    if (nb > 0) {
      const dim3 g1((unsigned)nb);
      switch (TQ) {
#define BMG_PANEL_COLS(NQv)                                                                                   \
  hipLaunchKernelGGL((k_panel_cols_lds<T, NQv>), g1, dim3(256), lds, s, TI, pa.n, q, Sp, pa.ldi,             \
                     values ? 1 : 0, pa.rows, X, ldx, coef, Out, ldo)
        case 1: BMG_PANEL_COLS(1); break;
        case 2: BMG_PANEL_COLS(2); break;
        case 3: BMG_PANEL_COLS(3); break;
        case 4: BMG_PANEL_COLS(4); break;
        default: BMG_PANEL_COLS(5); break;
#undef BMG_PANEL_COLS
      }
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_panel_xt<T>), dim3((unsigned)((pa.ldi * q + 255) / 256)), dim3(256), 0, s, pa.ldi, q,
                     pa.rows, X, ldx, Xt);
  const dim3 grid((unsigned)((pa.n + 63) / 64));
  if (TQ <= 4)
    hipLaunchKernelGGL((k_panel_cols<T, 4>), grid, dim3(256), 0, s, TI, pa.n, q, Sp, pa.ldi, values ? 1 : 0,
                       (const T *)Xt, coef, Out, ldo);
  else if (TQ <= 8)
    hipLaunchKernelGGL((k_panel_cols<T, 8>), grid, dim3(256), 0, s, TI, pa.n, q, Sp, pa.ldi, values ? 1 : 0,
                       (const T *)Xt, coef, Out, ldo);
  else
    hipLaunchKernelGGL((k_panel_cols<T, 12>), grid, dim3(256), 0, s, TI, pa.n, q, Sp, pa.ldi, values ? 1 : 0,
                       (const T *)Xt, coef, Out, ldo);
  return hipGetLastError();
}

// ------------------------------------------------------------------ set-up
// A[j][i] = NaN for every column j and panel slot i (padding slots included)
template <typename TA>
__global__ void k_panel_nan(int64_t cnt, TA *__restrict__ A) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * blockDim.x)
    A[e] = (TA)__builtin_nan("");
}
// then the observed values of panel row i = row rows[i] (one block per panel row)
__global__ __launch_bounds__(256) void k_panel_scatter(int ldi, const int32_t *__restrict__ rows,
                                                       const int64_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ idx,
                                                       const double *__restrict__ val, double *__restrict__ A,
                                                       float *__restrict__ A32) {
  const int i = blockIdx.x;
  const int64_t r = rows[i];
  for (int64_t p = ptr[r] + threadIdx.x; p < ptr[r + 1]; p += blockDim.x) {
    const int64_t o = (int64_t)idx[p] * ldi + i;
    A[o] = val[p];
    if (A32) A32[o] = (float)val[p];
  }
}
hipError_t launch_panel_fill(int P, int64_t n, int ldi, const int32_t *rows, const int64_t *ptr,
                             const int32_t *idx, const double *val, double *A, float *A32, hipStream_t s) {
  if (P <= 0) return hipSuccess;
  const int64_t cnt = n * ldi;
  hipLaunchKernelGGL((k_panel_nan<double>), dim3(4096), dim3(256), 0, s, cnt, A);
  if (A32) hipLaunchKernelGGL((k_panel_nan<float>), dim3(4096), dim3(256), 0, s, cnt, A32);
  hipLaunchKernelGGL(k_panel_scatter, dim3((unsigned)P), dim3(256), 0, s, ldi, rows, ptr, idx, val, A, A32);
  return hipGetLastError();
}

// keep[p] = 1 for the entries of a column-major orientation whose row is not
// in the panel (mask: 1 for panel rows)
__global__ void k_panel_keep(int64_t nnz, const int32_t *__restrict__ idx, const uint8_t *__restrict__ mask,
                             int32_t *__restrict__ keep) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnz) keep[p] = mask[idx[p]] ? 0 : 1;
}
// pos = exclusive prefix sum of keep; kept entries move to pos[p]; rptr[c] = pos[ptr[c]]
__global__ void k_panel_compact(int64_t nnz, const int32_t *__restrict__ keep, const int32_t *__restrict__ pos,
                                const int32_t *__restrict__ idx, const double *__restrict__ val,
                                int32_t *__restrict__ ridx, double *__restrict__ rval) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnz && keep[p]) {
    ridx[pos[p]] = idx[p];
    rval[pos[p]] = val[p];
  }
}
__global__ void k_panel_rptr(int64_t ncols, int64_t nnz, const int64_t *__restrict__ ptr,
                             const int32_t *__restrict__ keep, const int32_t *__restrict__ pos,
                             int64_t *__restrict__ rptr) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > ncols) return;
  const int64_t p = ptr[c];
  rptr[c] = p < nnz ? (int64_t)pos[p] : (nnz > 0 ? (int64_t)pos[nnz - 1] + keep[nnz - 1] : 0);
}
hipError_t launch_panel_keep(int64_t nnz, const int32_t *idx, const uint8_t *mask, int32_t *keep, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_panel_keep, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, idx, mask, keep);
  return hipGetLastError();
}
hipError_t launch_panel_compact(int64_t ncols, int64_t nnz, const int64_t *ptr, const int32_t *keep,
                                const int32_t *pos, const int32_t *idx, const double *val, int32_t *ridx,
                                double *rval, int64_t *rptr, hipStream_t s) {
  if (nnz > 0)
    hipLaunchKernelGGL(k_panel_compact, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, keep, pos,
                       idx, val, ridx, rval);
  hipLaunchKernelGGL(k_panel_rptr, dim3((unsigned)((ncols + 1 + 255) / 256)), dim3(256), 0, s, ncols, nnz, ptr,
                     keep, pos, rptr);
  return hipGetLastError();
}

template hipError_t launch_panel_resid<double>(const PanelArg<double> &, const double *, int, const double *, int,
                                               int, bool, bool, double *, int64_t, double *, double *,
                                               hipStream_t);
template hipError_t launch_panel_resid<float>(const PanelArg<float> &, const float *, int, const float *, int,
                                              int, bool, bool, double *, int64_t, double *, double *,
                                              hipStream_t);
template hipError_t launch_panel_rows<double>(const PanelArg<double> &, bool, const double *, int, int, double,
                                              const double *, int, int, const double *, int, double,
                                              const double *, int, double *, int, double *, int64_t, double *,
                                              int64_t, hipStream_t);
template hipError_t launch_panel_rows<float>(const PanelArg<float> &, bool, const float *, int, int, double,
                                             const float *, int, int, const float *, int, double, const float *,
                                             int, float *, int, double *, int64_t, double *, int64_t,
                                             hipStream_t);
template hipError_t launch_panel_cols<double>(const PanelArg<double> &, bool, const double *, int, int, double,
                                              double *, int, double *, hipStream_t);
template hipError_t launch_panel_cols<float>(const PanelArg<float> &, bool, const float *, int, int, double,
                                             float *, int, float *, hipStream_t);

}  // namespace bmg
