// Pair passes of the kernel-estimation QSDP (QSDP section; BM form eq. bm2):
// Omega is stored symmetrically (both (i, j) and (j, i), value d_ij^2) and the
// one factor W (n x k) is gathered on both sides.  One 64-lane wave per work
// unit of the rows plan; lanes stride over the entries and loop over the k
// columns; reductions in a fixed order, long rows summed piece by piece in
// piece order, so results are bitwise reproducible.  FP64 only.
#include <hip/hip_runtime.h>

#include "bmg_internal.h"
#include "units.h"

namespace bmg {

namespace {

constexpr int RK_WAVES = 4;  // waves per block

// r_p = ||w_i - w_j||^2 - d2_p (stored); per row deg_i = sum r, adeg_i = sum |r|;
// per block the partial sum of r^2.
__global__ __launch_bounds__(64 * RK_WAVES) void k_rke_res(Plan pl, const double *__restrict__ W, int ld,
                                                        int k, const double *__restrict__ d2,
                                                        double *__restrict__ r, double *__restrict__ deg,
                                                        double *__restrict__ adeg,
                                                        double *__restrict__ part,
                                                        double *__restrict__ bpart) {
  __shared__ double sm[RK_WAVES];
  const int64_t u = (int64_t)blockIdx.x * RK_WAVES + threadIdx.x / 64;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  double s = 0.0, sa = 0.0, s2 = 0.0;
  const bool live = u < pl.n_short + pl.n_pieces;
  Unit w{};
  if (live) {
    w = unit_of(pl, u);
    const double *wi = W + w.row * ld;
    for (int64_t e = w.beg + lane; e < w.end; e += 64) {
      const double *wj = W + (int64_t)pl.idx[e] * ld;
      double acc = 0.0;
      for (int c = 0; c < k; ++c) {
        const double d = wi[c] - wj[c];
        acc += d * d;
      }
      const double rr = acc - d2[e];
      r[e] = rr;
      s += rr;
      sa += fabs(rr);
      s2 += rr * rr;
    }
  }
  s = wave_sum64(s);
  sa = wave_sum64(sa);
  s2 = wave_sum64(s2);
  if (lane == 0) {
    sm[wv] = s2;
    if (live) {
      if (w.piece) {
        part[2 * w.p] = s;
        part[2 * w.p + 1] = sa;
      } else {
        deg[w.row] = s;
        adeg[w.row] = sa;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < RK_WAVES; ++q) t += sm[q];
    bpart[blockIdx.x] = t;
  }
}

__global__ void k_rke_fix(Plan pl, const double *__restrict__ part, double *__restrict__ deg,
                          double *__restrict__ adeg) {
  const int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= pl.n_long) return;
  double s = 0.0, sa = 0.0;
  for (int p = pl.long_p0[L]; p < pl.long_p0[L + 1]; ++p) {
    s += part[2 * p];
    sa += part[2 * p + 1];
  }
  deg[pl.long_rows[L]] = s;
  adeg[pl.long_rows[L]] = sa;
}

// Quartic coefficients along W + t D: per entry a1 = (w_i - w_j).(d_i - d_j),
// a2 = ||d_i - d_j||^2; per block sum r a1, a1^2, r a2, a1 a2, a2^2.
__global__ __launch_bounds__(64 * RK_WAVES) void k_rke_quartic(Plan pl, const double *__restrict__ W,
                                                            const double *__restrict__ D, int ld, int k,
                                                            const double *__restrict__ r,
                                                            double *__restrict__ bpart) {
  __shared__ double sm[RK_WAVES][5];
  const int64_t u = (int64_t)blockIdx.x * RK_WAVES + threadIdx.x / 64;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  if (u < pl.n_short + pl.n_pieces) {
    const Unit w = unit_of(pl, u);
    const double *wi = W + w.row * ld, *di = D + w.row * ld;
    for (int64_t e = w.beg + lane; e < w.end; e += 64) {
      const int64_t j = pl.idx[e];
      const double *wj = W + j * ld, *dj = D + j * ld;
      double a1 = 0.0, a2 = 0.0;
      for (int c = 0; c < k; ++c) {
        const double dd = di[c] - dj[c];
        a1 += (wi[c] - wj[c]) * dd;
        a2 += dd * dd;
      }
      const double rr = r[e];
      s0 += rr * a1;
      s1 += a1 * a1;
      s2 += rr * a2;
      s3 += a1 * a2;
      s4 += a2 * a2;
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
    for (int q = 0; q < RK_WAVES; ++q) t += sm[q][threadIdx.x];
    bpart[(int64_t)blockIdx.x * 5 + threadIdx.x] = t;
  }
}

// out[c] = sum over b of parts[b * nc + c], one block, fixed order.
__global__ __launch_bounds__(256) void k_sum_parts(const double *__restrict__ parts, int64_t nb, int nc,
                                                   double *__restrict__ out) {
  __shared__ double sm[4][8];
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  for (int c = 0; c < nc; ++c) {
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += 256) v += parts[b * nc + c];
    v = wave_sum64(v);
    if (lane == 0) sm[wv][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < nc) out[threadIdx.x] = sm[0][threadIdx.x] + sm[1][threadIdx.x] + sm[2][threadIdx.x] +
                                           sm[3][threadIdx.x];
}

// Out[i, c] = deg[i] U[i, c] - Out[i, c]
__global__ void k_rowscale_sub(int64_t n, int q, const double *__restrict__ deg,
                               const double *__restrict__ U, int ldu, double *__restrict__ Out, int ldo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * q) return;
  const int64_t i = t / q;
  const int c = (int)(t % q);
  Out[i * ldo + c] = deg[i] * U[i * ldu + c] - Out[i * ldo + c];
}

// Column means in two steps, fixed order: block b sums rows [b R, (b + 1) R)
// of every column (consecutive threads read consecutive columns), then each
// element subtracts its column's mean, summed from the NB partials in order.
constexpr int CC_BLOCKS = 64;
// grid (CC_BLOCKS, ceil(q / 64)): a block covers one row chunk and up to 64
// columns; its 256 threads split the chunk's rows nr ways per column and
// combine the nr sums in order through LDS.
__global__ __launch_bounds__(256) void k_colsum_part(int64_t n, int q, const double *__restrict__ V, int ld,
                                                     double *__restrict__ part) {
  __shared__ double sm[256];
  const int64_t R = (n + CC_BLOCKS - 1) / CC_BLOCKS;
  const int64_t i0 = (int64_t)blockIdx.x * R, i1 = i0 + R < n ? i0 + R : n;
  const int c0 = blockIdx.y * 64, qt = q - c0 < 64 ? q - c0 : 64, nr = 256 / qt;
  const int r = threadIdx.x / qt, cc = threadIdx.x % qt;
  double v = 0.0;
  if (r < nr)
    for (int64_t i = i0 + r; i < i1; i += nr) v += V[i * ld + c0 + cc];
  sm[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < qt) {
    double t = 0.0;
    for (int rr = 0; rr < nr; ++rr) t += sm[rr * qt + threadIdx.x];
    part[(int64_t)blockIdx.x * q + c0 + threadIdx.x] = t;
  }
}
__global__ void k_colmean_sub(int64_t n, int q, double *__restrict__ V, int ld,
                              const double *__restrict__ part) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * q) return;
  const int64_t i = t / q;
  const int c = (int)(t % q);
  double sum = 0.0;
  for (int b = 0; b < CC_BLOCKS; ++b) sum += part[(int64_t)b * q + c];
  V[i * ld + c] -= sum / (double)n;
}

// Frobenius inner products <A_j, B_j> of np pairs of n x k matrices (ld):
// per block partial sums (block b covers rows b, b + grid, ...), fixed order.
struct DotPairs {
  const double *A[4];
  const double *B[4];
};
__global__ __launch_bounds__(256) void k_frob_dots(int64_t n, int k, int ld, DotPairs dp, int np,
                                                   double *__restrict__ bpart) {
  __shared__ double sm[4][4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t tot = n * (int64_t)k, stride = (int64_t)gridDim.x * 256;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < tot; t += stride) {
    const int64_t i = t / k, c = t % k, o = i * ld + c;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < np) v[j] += dp.A[j][o] * dp.B[j][o];
  }
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const double t = wave_sum64(v[j]);
    if (lane == 0) sm[wv][j] = t;
  }
  __syncthreads();
  if (threadIdx.x < np)
    bpart[(int64_t)blockIdx.x * np + threadIdx.x] =
        sm[0][threadIdx.x] + sm[1][threadIdx.x] + sm[2][threadIdx.x] + sm[3][threadIdx.x];
}

// flag = 1 when the two orientations differ (the pattern or values are not symmetric)
__global__ void k_cmp_orient(int64_t nnz, const int32_t *__restrict__ a, const int32_t *__restrict__ b,
                             const double *__restrict__ va, const double *__restrict__ vb,
                             int *__restrict__ flag) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz && (a[e] != b[e] || va[e] != vb[e])) flag[0] = 1;
}

}  // namespace

hipError_t launch_rke_res(const Plan &pl, const double *W, int ld, int k, const double *d2, double *r,
                          double *deg, double *adeg, double *part, double *bpart, int64_t bpart_cap,
                          double *out, hipStream_t s) {
  const int64_t units = pl.n_short + pl.n_pieces;
  const int64_t nb = (units + RK_WAVES - 1) / RK_WAVES;
  if (nb > bpart_cap) return hipErrorInvalidValue;
  if (nb > 0)
    hipLaunchKernelGGL(k_rke_res, dim3((unsigned)nb), dim3(64 * RK_WAVES), 0, s, pl, W, ld, k, d2, r, deg,
                       adeg, part, bpart);
  if (pl.n_long > 0)
    hipLaunchKernelGGL(k_rke_fix, dim3((unsigned)((pl.n_long + 255) / 256)), dim3(256), 0, s, pl,
                       (const double *)part, deg, adeg);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, (const double *)bpart, nb, 1, out);
  return hipGetLastError();
}

hipError_t launch_rke_quartic(const Plan &pl, const double *W, const double *D, int ld, int k,
                              const double *r, double *bpart, int64_t bpart_cap, double *out,
                              hipStream_t s) {
  const int64_t units = pl.n_short + pl.n_pieces;
  const int64_t nb = (units + RK_WAVES - 1) / RK_WAVES;
  if (nb * 5 > bpart_cap) return hipErrorInvalidValue;
  if (nb > 0)
    hipLaunchKernelGGL(k_rke_quartic, dim3((unsigned)nb), dim3(64 * RK_WAVES), 0, s, pl, W, D, ld, k, r,
                       bpart);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, (const double *)bpart, nb, 5, out);
  return hipGetLastError();
}

hipError_t launch_frob_dots(int64_t n, int k, int ld, const double *const *A, const double *const *B, int np,
                            double *bpart, double *out, hipStream_t s) {
  constexpr int NB = 128;
  if (np < 1 || np > 4) return hipErrorInvalidValue;
  DotPairs dp{};
  for (int j = 0; j < np; ++j) {
    dp.A[j] = A[j];
    dp.B[j] = B[j];
  }
  hipLaunchKernelGGL(k_frob_dots, dim3(NB), dim3(256), 0, s, n, k, ld, dp, np, bpart);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, (const double *)bpart, (int64_t)NB, np, out);
  return hipGetLastError();
}

hipError_t launch_rowscale_sub(int64_t n, int q, const double *deg, const double *U, int ldu, double *Out,
                               int ldo, hipStream_t s) {
  const int64_t tot = n * (int64_t)q;
  if (tot > 0)
    hipLaunchKernelGGL(k_rowscale_sub, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, q, deg, U,
                       ldu, Out, ldo);
  return hipGetLastError();
}

hipError_t launch_center_cols(int64_t n, int q, double *V, int ld, double *part, int64_t part_cap,
                              hipStream_t s) {
  if (n <= 0 || q <= 0) return hipSuccess;
  if ((int64_t)CC_BLOCKS * q > part_cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_colsum_part, dim3(CC_BLOCKS, (unsigned)((q + 63) / 64)), dim3(256), 0, s, n, q,
                     (const double *)V, ld, part);
  const int64_t tot = n * (int64_t)q;
  hipLaunchKernelGGL(k_colmean_sub, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, q, V, ld,
                     (const double *)part);
  return hipGetLastError();
}

hipError_t launch_cmp_orient(int64_t nnz, const int32_t *a, const int32_t *b, const double *va,
                             const double *vb, int *flag, hipStream_t s) {
  if (nnz > 0)
    hipLaunchKernelGGL(k_cmp_orient, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, a, b, va,
                       vb, flag);
  return hipGetLastError();
}

}  // namespace bmg
