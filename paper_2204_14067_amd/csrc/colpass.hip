// Column passes of the polyMF-SS BM solver (block coordinate descent over the
// column pairs (w_j, h_j) with an exact quartic line search, Sec. 6.1.1).
//
// Work units are the rows of one orientation of Omega as the load-balancing
// plan splits them: unit u < n_short is a short row, unit n_short + p is
// piece p of a long row.  One 64-lane wave per unit; lanes stride over the
// unit's entries, the wave reduces in a fixed order and long rows are summed
// piece by piece in piece order, so every result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "bmg_internal.h"
#include "units.h"

namespace bmg {

namespace {

constexpr int CP_WAVES = 4;  // waves per block

// One orientation.  Gown holds one record per row of this orientation, Goth
// one per gathered index (Q4 layout: prev, step, x, dir):
//  * upd: r += s_row y'_l + x'_row s_l - s_row s_l, with x' / y' the values of
//    the block just stepped (already moved by s) on each side;
//  * nxt: g = sum r y_l, c = sum y_l^2 over the row (y = the block's current
//    value on the gathered side), and the direction
//    dir = -(g + lam x_row) / (c + lam) goes to Gown[row].w.
template <typename T>
__global__ __launch_bounds__(64 * CP_WAVES) void k_col_grad(Plan pl, T *__restrict__ r,
                                                         Q4<T> *__restrict__ Gown,
                                                         const Q4<T> *__restrict__ Goth, int upd,
                                                         int nxt, double lam,
                                                         double *__restrict__ part) {
  const int64_t u = (int64_t)blockIdx.x * CP_WAVES + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (u >= pl.n_short + pl.n_pieces) return;
  const Unit w = unit_of(pl, u);
  const Q4<T> own = Gown[w.row];
  const double xp = (double)own.x, so = (double)own.y;
  double g = 0.0, c = 0.0;
  for (int64_t e = w.beg + lane; e < w.end; e += 64) {
    const Q4<T> ot = Goth[pl.idx[e]];
    double rr = (double)r[e];
    if (upd) {
      const double yp = (double)ot.x, sl = (double)ot.y;
      rr += so * yp + xp * sl - so * sl;
      r[e] = (T)rr;
      rr = (double)r[e];
    }
    const double y = (double)ot.z;
    g += rr * y;
    c += y * y;
  }
  if (!nxt) return;
  g = wave_sum64(g);
  c = wave_sum64(c);
  if (lane != 0) return;
  if (w.piece) {
    part[2 * w.p] = g;
    part[2 * w.p + 1] = c;
  } else {
    Gown[w.row].w = (T)(-(g + lam * (double)own.z) / (c + lam));
  }
}

// Long rows: sum the pieces' (g, c) in piece order, then the direction.
template <typename T>
__global__ void k_col_fix(Plan pl, const double *__restrict__ part, double lam,
                          Q4<T> *__restrict__ Gown) {
  const int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= pl.n_long) return;
  double g = 0.0, c = 0.0;
  for (int p = pl.long_p0[L]; p < pl.long_p0[L + 1]; ++p) {
    g += part[2 * p];
    c += part[2 * p + 1];
  }
  const int64_t row = pl.long_rows[L];
  Gown[row].w = (T)(-(g + lam * (double)Gown[row].z) / (c + lam));
}

// Coefficient sums of the quartic along (w + t dw, h + t dh) on the rows
// orientation: with a = dw_i h_l + w_i dh_l and b = dw_i dh_l per entry,
// per block: sum r a, sum a^2, sum r b, sum a b, sum b^2.
constexpr int DOT_BLOCKS = 128;

template <typename T>
__device__ void col_dots_block(int64_t m, int64_t n, const Q4<T> *__restrict__ Gm,
                               const Q4<T> *__restrict__ Gn, double *__restrict__ dpart, int bid);

// Blocks 0..nbq-1: the quartic sums of nbq x CP_WAVES work units; blocks
// nbq..nbq+DOT_BLOCKS-1: the record dot products (col_dots_block).
template <typename T>
__global__ __launch_bounds__(64 * CP_WAVES) void k_col_quartic(Plan pl, const T *__restrict__ r,
                                                            const Q4<T> *__restrict__ Gm,
                                                            const Q4<T> *__restrict__ Gn,
                                                            double *__restrict__ bpart, int64_t nbq,
                                                            int64_t m, int64_t n,
                                                            double *__restrict__ dpart) {
  if ((int64_t)blockIdx.x >= nbq) {
    col_dots_block<T>(m, n, Gm, Gn, dpart, (int)(blockIdx.x - nbq));
    return;
  }
  __shared__ double sm[CP_WAVES][5];
  const int64_t u = (int64_t)blockIdx.x * CP_WAVES + threadIdx.x / 64;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  if (u < pl.n_short + pl.n_pieces) {
    const Unit w = unit_of(pl, u);
    const Q4<T> own = Gm[w.row];
    const double x = (double)own.z, dx = (double)own.w;
    for (int64_t e = w.beg + lane; e < w.end; e += 64) {
      const Q4<T> ot = Gn[pl.idx[e]];
      const double y = (double)ot.z, dy = (double)ot.w, rr = (double)r[e];
      const double a = dx * y + x * dy, b = dx * dy;
      s0 += rr * a;
      s1 += a * a;
      s2 += rr * b;
      s3 += a * b;
      s4 += b * b;
    }
  }
  s0 = wave_sum64(s0);
  s1 = wave_sum64(s1);
  s2 = wave_sum64(s2);
  s3 = wave_sum64(s3);
  s4 = wave_sum64(s4);
  if (lane == 0) {
    sm[wv][0] = s0; sm[wv][1] = s1; sm[wv][2] = s2; sm[wv][3] = s3; sm[wv][4] = s4;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double t = 0.0;
    for (int q = 0; q < CP_WAVES; ++q) t += sm[q][threadIdx.x];
    bpart[(int64_t)blockIdx.x * 5 + threadIdx.x] = t;
  }
}

// Dot block b of DOT_BLOCKS: sum x d, sum d^2 over its slice of the m records
// and of the n records (x = the block's current value, d = its direction).
template <typename T>
__device__ void col_dots_block(int64_t m, int64_t n, const Q4<T> *__restrict__ Gm,
                               const Q4<T> *__restrict__ Gn, double *__restrict__ dpart, int bid) {
  __shared__ double sm[4][4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)DOT_BLOCKS * 256;
  for (int64_t i = (int64_t)bid * 256 + threadIdx.x; i < m; i += stride) {
    const Q4<T> g = Gm[i];
    v[0] += (double)g.z * (double)g.w;
    v[1] += (double)g.w * (double)g.w;
  }
  for (int64_t i = (int64_t)bid * 256 + threadIdx.x; i < n; i += stride) {
    const Q4<T> g = Gn[i];
    v[2] += (double)g.z * (double)g.w;
    v[3] += (double)g.w * (double)g.w;
  }
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double t = wave_sum64(v[q]);
    if (lane == 0) sm[wv][q] = t;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const double t = sm[0][threadIdx.x] + sm[1][threadIdx.x] + sm[2][threadIdx.x] + sm[3][threadIdx.x];
    dpart[bid * 4 + threadIdx.x] = t;
  }
}

// The step of the block from its quartic's sums h (one thread): state[0] =
// t, state[1] counts the blocks with t > 0, state[2] = 1 on a non-finite
// coefficient (t = 0 then).
__device__ void col_step_of(const double *h, double lam, double *__restrict__ state) {
  const double c1 = h[0] + lam * (h[5] + h[7]);
  const double c2 = 0.5 * h[1] + h[2] + 0.5 * lam * (h[6] + h[8]);
  const double c3 = h[3], c4 = 0.5 * h[4];
  double t = 0.0;
  if (isfinite(c1) && isfinite(c2) && isfinite(c3) && isfinite(c4)) t = quartic_min(c1, c2, c3, c4);
  else state[2] = 1.0;
  state[0] = t;
  if (t > 0.0) state[1] += 1.0;
}

// out[0..4]: the quartic sums over nb blocks; out[5..8]: the four dot
// products; with state, also the block's step (col_step_of).
__global__ __launch_bounds__(256) void k_col_reduce(const double *__restrict__ bpart, int64_t nb,
                                                    const double *__restrict__ dpart,
                                                    double *__restrict__ out, double lam,
                                                    double *__restrict__ state) {
  __shared__ double sm[4][9];
  double v[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) v[q] = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += 256)
#pragma unroll
    for (int q = 0; q < 5; ++q) v[q] += bpart[b * 5 + q];
  for (int b = threadIdx.x; b < DOT_BLOCKS; b += 256)
#pragma unroll
    for (int q = 0; q < 4; ++q) v[5 + q] += dpart[b * 4 + q];
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const double t = wave_sum64(v[q]);
    if (lane == 0) sm[wv][q] = t;
  }
  __syncthreads();
  if (threadIdx.x < 9) out[threadIdx.x] = sm[0][threadIdx.x] + sm[1][threadIdx.x] + sm[2][threadIdx.x] +
                                          sm[3][threadIdx.x];
  if (state && threadIdx.x == 0) {
    double h[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) h[q] = sm[0][q] + sm[1][q] + sm[2][q] + sm[3][q];
    col_step_of(h, lam, state);
  }
}

// Block j moves by t along its direction (t = 0: no move) and the records
// are rewritten for block jn (jn < 0: none):
//   G[i] = {x_i + t d_i, t d_i, X[i, jn], 0},  X[i, j] = x_i + t d_i.
template <typename T>
__global__ void k_col_step(int64_t m, int64_t n, T *__restrict__ W, T *__restrict__ H, int ld, int j,
                           int jn, const double *__restrict__ tp, Q4<T> *__restrict__ Gm,
                           Q4<T> *__restrict__ Gn) {
  const double t = *tp;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    const Q4<T> g = Gm[i];
    const T s = (T)(t * (double)g.w);
    const T x = g.z + s;
    if (t != 0.0) W[i * ld + j] = x;
    Gm[i] = Q4<T>{x, s, jn >= 0 ? W[i * ld + jn] : (T)0, (T)0};
  }
  if (i < n) {
    const Q4<T> g = Gn[i];
    const T s = (T)(t * (double)g.w);
    const T x = g.z + s;
    if (t != 0.0) H[i * ld + j] = x;
    Gn[i] = Q4<T>{x, s, jn >= 0 ? H[i * ld + jn] : (T)0, (T)0};
  }
}

// Records for the first block: {0, 0, X[i, 0], 0}.
template <typename T>
__global__ void k_col_pack0(int64_t m, int64_t n, const T *__restrict__ W, const T *__restrict__ H,
                            int ld, Q4<T> *__restrict__ Gm, Q4<T> *__restrict__ Gn) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) Gm[i] = Q4<T>{(T)0, (T)0, W[i * ld], (T)0};
  if (i < n) Gn[i] = Q4<T>{(T)0, (T)0, H[i * ld], (T)0};
}

}  // namespace

template <typename T>
hipError_t launch_col_pack0(int64_t m, int64_t n, const T *W, const T *H, int ld, Q4<T> *Gm, Q4<T> *Gn,
                            hipStream_t s) {
  const int64_t mx = m > n ? m : n;
  if (mx > 0)
    hipLaunchKernelGGL((k_col_pack0<T>), dim3((unsigned)((mx + 255) / 256)), dim3(256), 0, s, m, n, W, H,
                       ld, Gm, Gn);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col_grad(const Plan &pl, T *r, Q4<T> *Gown, const Q4<T> *Goth, bool upd, double lam,
                           double *part, hipStream_t s) {
  const int64_t units = pl.n_short + pl.n_pieces;
  if (units > 0) {
    const int64_t nb = (units + CP_WAVES - 1) / CP_WAVES;
    hipLaunchKernelGGL((k_col_grad<T>), dim3((unsigned)nb), dim3(64 * CP_WAVES), 0, s, pl, r, Gown, Goth,
                       upd ? 1 : 0, 1, lam, part);
  }
  if (pl.n_long > 0)
    hipLaunchKernelGGL((k_col_fix<T>), dim3((unsigned)((pl.n_long + 255) / 256)), dim3(256), 0, s, pl,
                       (const double *)part, lam, Gown);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col_quartic(const Plan &pl, const T *r, int64_t m, int64_t n, const Q4<T> *Gm,
                              const Q4<T> *Gn, double *bpart, int64_t bpart_cap, double *dpart,
                              double *out, double lam, double *state, hipStream_t s) {
  const int64_t units = pl.n_short + pl.n_pieces;
  const int64_t nb = (units + CP_WAVES - 1) / CP_WAVES;
  if (nb * 5 > bpart_cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_col_quartic<T>), dim3((unsigned)(nb + DOT_BLOCKS)), dim3(64 * CP_WAVES), 0, s, pl,
                     r, Gm, Gn, bpart, nb, m, n, dpart);
  hipLaunchKernelGGL(k_col_reduce, dim3(1), dim3(256), 0, s, (const double *)bpart, nb,
                     (const double *)dpart, out, lam, state);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col_step(int64_t m, int64_t n, T *W, T *H, int ld, int j, int jn, const double *tp,
                           Q4<T> *Gm, Q4<T> *Gn, hipStream_t s) {
  const int64_t mx = m > n ? m : n;
  if (mx > 0)
    hipLaunchKernelGGL((k_col_step<T>), dim3((unsigned)((mx + 255) / 256)), dim3(256), 0, s, m, n, W, H,
                       ld, j, jn, tp, Gm, Gn);
  return hipGetLastError();
}

#define BMG_INST_COL(T)                                                                            \
  template hipError_t launch_col_pack0<T>(int64_t, int64_t, const T *, const T *, int, Q4<T> *,     \
                                          Q4<T> *, hipStream_t);                                    \
  template hipError_t launch_col_grad<T>(const Plan &, T *, Q4<T> *, const Q4<T> *, bool, double,   \
                                         double *, hipStream_t);                                    \
  template hipError_t launch_col_quartic<T>(const Plan &, const T *, int64_t, int64_t,              \
                                            const Q4<T> *, const Q4<T> *, double *, int64_t,        \
                                            double *, double *, double, double *, hipStream_t);                       \
  template hipError_t launch_col_step<T>(int64_t, int64_t, T *, T *, int, int, int, const double *, Q4<T> *, \
                                         Q4<T> *, hipStream_t);
BMG_INST_COL(double)
BMG_INST_COL(float)

}  // namespace bmg
