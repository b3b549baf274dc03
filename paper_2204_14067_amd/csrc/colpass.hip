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

namespace bmg {

namespace {

constexpr int CP_WAVES = 4;  // waves per block

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct Unit {
  int64_t row, beg, end;
  bool piece;
  int64_t p;
};

__device__ __forceinline__ Unit unit_of(const Plan &pl, int64_t u) {
  Unit x;
  if (u < pl.n_short) {
    x.row = pl.short_rows[u];
    x.beg = pl.ptr[x.row];
    x.end = pl.ptr[x.row + 1];
    x.piece = false;
    x.p = -1;
  } else {
    x.p = u - pl.n_short;
    x.row = pl.piece_row[x.p];
    x.beg = pl.piece_beg[x.p];
    x.end = pl.piece_end[x.p];
    x.piece = true;
  }
  return x;
}

// One orientation: own-side factor X (rows of this orientation), gathered
// factor Y (indexed by idx), both at leading dimension ld.
//  * upd: r += su[row] y'_l + x'_row sv[l] - su[row] sv[l] with x' = X[:, jp],
//    y' = Y[:, jp] (the block jp just stepped by su, sv, already applied to X, Y)
//  * next (jn >= 0): g = sum r y_l, c = sum y_l^2 with y = Y[:, jn]; the
//    direction dir[row] = -(g + lam x_row) / (c + lam), x = X[:, jn]
template <typename T>
__global__ __launch_bounds__(64 * CP_WAVES) void k_col_grad(Plan pl, T *__restrict__ r,
                                                         const T *__restrict__ X,
                                                         const T *__restrict__ Y, int ld, int jp,
                                                         const T *__restrict__ su,
                                                         const T *__restrict__ sv, int jn,
                                                         double lam, T *__restrict__ dir,
                                                         double *__restrict__ part) {
  const int64_t u = (int64_t)blockIdx.x * CP_WAVES + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (u >= pl.n_short + pl.n_pieces) return;
  const Unit w = unit_of(pl, u);
  const bool upd = jp >= 0, nxt = jn >= 0;
  double ux = 0.0, xp = 0.0;
  if (upd) {
    ux = (double)su[w.row];
    xp = (double)X[w.row * ld + jp];
  }
  double g = 0.0, c = 0.0;
  for (int64_t e = w.beg + lane; e < w.end; e += 64) {
    const int64_t l = pl.idx[e];
    double rr = (double)r[e];
    if (upd) {
      const double yp = (double)Y[l * ld + jp], vl = (double)sv[l];
      rr += ux * yp + xp * vl - ux * vl;
      r[e] = (T)rr;
      rr = (double)r[e];
    }
    if (nxt) {
      const double y = (double)Y[l * ld + jn];
      g += rr * y;
      c += y * y;
    }
  }
  if (!nxt) return;
  g = wave_sum64(g);
  c = wave_sum64(c);
  if (lane != 0) return;
  if (w.piece) {
    part[2 * w.p] = g;
    part[2 * w.p + 1] = c;
  } else {
    const double x = (double)X[w.row * ld + jn];
    dir[w.row] = (T)(-(g + lam * x) / (c + lam));
  }
}

// Long rows: sum the pieces' (g, c) in piece order, then the direction.
template <typename T>
__global__ void k_col_fix(Plan pl, const double *__restrict__ part, const T *__restrict__ X, int ld,
                          int jn, double lam, T *__restrict__ dir) {
  const int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= pl.n_long) return;
  double g = 0.0, c = 0.0;
  for (int p = pl.long_p0[L]; p < pl.long_p0[L + 1]; ++p) {
    g += part[2 * p];
    c += part[2 * p + 1];
  }
  const int64_t row = pl.long_rows[L];
  dir[row] = (T)(-(g + lam * (double)X[row * ld + jn]) / (c + lam));
}

// Coefficient sums of the quartic along (w + t dw, h + t dh) on the rows
// orientation: with a = dw_i h_l + w_i dh_l and b = dw_i dh_l per entry,
// per block: sum r a, sum a^2, sum r b, sum a b, sum b^2.
template <typename T>
__global__ __launch_bounds__(64 * CP_WAVES) void k_col_quartic(Plan pl, const T *__restrict__ r,
                                                            const T *__restrict__ W,
                                                            const T *__restrict__ H, int ld, int j,
                                                            const T *__restrict__ dw,
                                                            const T *__restrict__ dh,
                                                            double *__restrict__ bpart) {
  __shared__ double sm[CP_WAVES][5];
  const int64_t u = (int64_t)blockIdx.x * CP_WAVES + threadIdx.x / 64;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  if (u < pl.n_short + pl.n_pieces) {
    const Unit w = unit_of(pl, u);
    const double x = (double)W[w.row * ld + j], dx = (double)dw[w.row];
    for (int64_t e = w.beg + lane; e < w.end; e += 64) {
      const int64_t l = pl.idx[e];
      const double y = (double)H[l * ld + j], dy = (double)dh[l], rr = (double)r[e];
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

constexpr int DOT_BLOCKS = 128;

// Per block b: sum w dw, sum dw^2 over its slice of the m rows and
// sum h dh, sum dh^2 over its slice of the n rows.
template <typename T>
__global__ __launch_bounds__(256) void k_col_dots(int64_t m, int64_t n, const T *__restrict__ W,
                                                  const T *__restrict__ H, int ld, int j,
                                                  const T *__restrict__ dw,
                                                  const T *__restrict__ dh,
                                                  double *__restrict__ dpart) {
  __shared__ double sm[4][4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += stride) {
    const double d = (double)dw[i];
    v[0] += (double)W[i * ld + j] * d;
    v[1] += d * d;
  }
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const double d = (double)dh[i];
    v[2] += (double)H[i * ld + j] * d;
    v[3] += d * d;
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
    dpart[blockIdx.x * 4 + threadIdx.x] = t;
  }
}

// out[0..4]: the quartic sums over nb blocks; out[5..8]: the four dot products.
__global__ __launch_bounds__(256) void k_col_reduce(const double *__restrict__ bpart, int64_t nb,
                                                    const double *__restrict__ dpart,
                                                    double *__restrict__ out) {
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
}

// su = t dw, sv = t dh; W[:, j] += su, H[:, j] += sv.
template <typename T>
__global__ void k_col_step(int64_t m, int64_t n, T *__restrict__ W, T *__restrict__ H, int ld, int j,
                           const T *__restrict__ dw, const T *__restrict__ dh, double t,
                           T *__restrict__ su, T *__restrict__ sv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    const T s = (T)(t * (double)dw[i]);
    su[i] = s;
    W[i * ld + j] += s;
  }
  if (i < n) {
    const T s = (T)(t * (double)dh[i]);
    sv[i] = s;
    H[i * ld + j] += s;
  }
}

}  // namespace

template <typename T>
hipError_t launch_col_grad(const Plan &pl, T *r, const T *X, const T *Y, int ld, int jp, const T *su,
                           const T *sv, int jn, double lam, T *dir, double *part, hipStream_t s) {
  const int64_t units = pl.n_short + pl.n_pieces;
  if (units > 0) {
    const int64_t nb = (units + CP_WAVES - 1) / CP_WAVES;
    hipLaunchKernelGGL((k_col_grad<T>), dim3((unsigned)nb), dim3(64 * CP_WAVES), 0, s, pl, r, X, Y, ld,
                       jp, su, sv, jn, lam, dir, part);
  }
  if (jn >= 0 && pl.n_long > 0)
    hipLaunchKernelGGL((k_col_fix<T>), dim3((unsigned)((pl.n_long + 255) / 256)), dim3(256), 0, s, pl,
                       (const double *)part, X, ld, jn, lam, dir);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col_quartic(const Plan &pl, const T *r, int64_t m, int64_t n, const T *W,
                              const T *H, int ld, int j, const T *dw, const T *dh, double *bpart,
                              int64_t bpart_cap, double *dpart, double *out, hipStream_t s) {
  const int64_t units = pl.n_short + pl.n_pieces;
  const int64_t nb = (units + CP_WAVES - 1) / CP_WAVES;
  if (nb * 5 > bpart_cap) return hipErrorInvalidValue;
  if (nb > 0)
    hipLaunchKernelGGL((k_col_quartic<T>), dim3((unsigned)nb), dim3(64 * CP_WAVES), 0, s, pl, r, W, H,
                       ld, j, dw, dh, bpart);
  hipLaunchKernelGGL((k_col_dots<T>), dim3(DOT_BLOCKS), dim3(256), 0, s, m, n, W, H, ld, j, dw, dh,
                     dpart);
  hipLaunchKernelGGL(k_col_reduce, dim3(1), dim3(256), 0, s, (const double *)bpart, nb,
                     (const double *)dpart, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col_step(int64_t m, int64_t n, T *W, T *H, int ld, int j, const T *dw, const T *dh,
                           double t, T *su, T *sv, hipStream_t s) {
  const int64_t mx = m > n ? m : n;
  if (mx > 0)
    hipLaunchKernelGGL((k_col_step<T>), dim3((unsigned)((mx + 255) / 256)), dim3(256), 0, s, m, n, W, H,
                       ld, j, dw, dh, t, su, sv);
  return hipGetLastError();
}

#define BMG_INST_COL(T)                                                                            \
  template hipError_t launch_col_grad<T>(const Plan &, T *, const T *, const T *, int, int,         \
                                         const T *, const T *, int, double, T *, double *,         \
                                         hipStream_t);                                              \
  template hipError_t launch_col_quartic<T>(const Plan &, const T *, int64_t, int64_t, const T *,  \
                                            const T *, int, int, const T *, const T *, double *,   \
                                            int64_t, double *, double *, hipStream_t);              \
  template hipError_t launch_col_step<T>(int64_t, int64_t, T *, T *, int, int, const T *, const T *, \
                                         double, T *, T *, hipStream_t);
BMG_INST_COL(double)
BMG_INST_COL(float)

}  // namespace bmg
