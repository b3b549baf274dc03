// HIP kernels for gfx950 (CDNA4, wave64) of the BM-Global matrix-completion
// hot path other than the row kernels of the sparse passes (rowpass.h):
// scalar reductions, tall-skinny Gram on FP64 matrix cores, tall x small
// products, elementwise kernels, the counter RNG and problem set-up.
#include <hip/hip_runtime.h>

#include "rowpass.h"

namespace bmg {

// Offsets (from the row start) of the first entry of each long row at or
// beyond each column-range boundary: out[i * (nr + 1) + k] for boundary k * wc.
__global__ void k_range_bounds(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                               const int32_t *__restrict__ rows, int64_t n, int nr, int64_t wc,
                               int32_t *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * (nr + 1)) return;
  const int64_t i = t / (nr + 1);
  const int kb = (int)(t % (nr + 1));
  const int row = rows[i];
  int64_t b = ptr[row], e = ptr[row + 1];
  const int64_t b0 = b, c = (int64_t)kb * wc;
  while (b < e) {
    const int64_t mid = (b + e) >> 1;
    if (idx[mid] < c) b = mid + 1; else e = mid;
  }
  out[t] = (int32_t)(b - b0);
}
hipError_t launch_range_bounds(const int64_t *ptr, const int32_t *idx, const int32_t *rows,
                               int64_t n, int nr, int64_t wc, int32_t *out, hipStream_t s) {
  const int64_t t = n * (nr + 1);
  if (t == 0) return hipSuccess;
  hipLaunchKernelGGL(k_range_bounds, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, ptr, idx,
                     rows, n, nr, wc, out);
  return hipGetLastError();
}

// ============================================================================ scalar reduction
// Sums nsum interleaved per-wave partials in a fixed order.  Stage 1: block c
// takes a contiguous run of waves; thread t adds waves t, t+256, ... of the run
// in increasing order, then a fixed binary tree; stage 2 does the same over
// the stage-1 sums in one block.
constexpr int WSUM_BLOCKS = 256;

__global__ __launch_bounds__(256) void k_reduce_wsum(const double *__restrict__ wsum,
                                                     int64_t waves, int nsum, int64_t run,
                                                     double *__restrict__ out) {
  __shared__ double sh[256];
  const int64_t w0 = (int64_t)blockIdx.x * run;
  int64_t w1 = w0 + run;
  if (w1 > waves) w1 = waves;
  for (int c = 0; c < nsum; ++c) {
    double s = 0.0;
    for (int64_t w = w0 + threadIdx.x; w < w1; w += 256) s += wsum[w * nsum + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)blockIdx.x * nsum + c] = sh[0];
    __syncthreads();
  }
}

hipError_t launch_reduce_wsum(const double *wsum, int64_t waves, int nsum, double *tmp,
                              double *out, hipStream_t s) {
  int64_t nb = (waves + 1023) / 1024;   // >= 1024 waves per stage-1 block
  if (nb > WSUM_BLOCKS) nb = WSUM_BLOCKS;
  if (nb <= 1) {
    hipLaunchKernelGGL(k_reduce_wsum, dim3(1), dim3(256), 0, s, wsum, waves, nsum, waves, out);
    return hipGetLastError();
  }
  const int64_t run = (waves + nb - 1) / nb;
  nb = (waves + run - 1) / run;
  hipLaunchKernelGGL(k_reduce_wsum, dim3((unsigned)nb), dim3(256), 0, s, wsum, waves, nsum, run,
                     tmp);
  hipLaunchKernelGGL(k_reduce_wsum, dim3(1), dim3(256), 0, s, (const double *)tmp, nb, nsum, nb,
                     out);
  return hipGetLastError();
}

// ============================================================================ tall-skinny Gram
// out[a x b] = X[N x a]^T Y[N x b] with FP64 matrix cores (16x16x4 FP64 MFMA).
// Row block c of the grid covers rows [c rpb, (c+1) rpb); blockIdx.y picks a
// group of up to 4 x 4 output tiles of 16 x 16.  The four waves of a block
// take the block's 4-row steps in turn; each lane loads its fragment values
// straight from memory: lane l holds X[r + l/16][16 t + l%16] (A operand,
// k = l/16) and Y[r + l/16][16 u + l%16] (B operand), so one load covers four
// rows x 128 bytes.  The waves' accumulators are added in wave order through
// LDS into part[c][a][b]; k_gram_reduce then adds the row blocks in order.
typedef double d4_t __attribute__((ext_vector_type(4)));

template <typename T>
__global__ __launch_bounds__(256) void k_gram(int64_t N, int a, const T *__restrict__ X, int ldx,
                                              int b, const T *__restrict__ Y, int ldy,
                                              int64_t rpb, double *__restrict__ part) {
  __shared__ double red[4][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int TA = (a + 15) / 16, TB = (b + 15) / 16, ngj = (TB + 3) / 4;
  const int ta0 = 4 * (blockIdx.y / ngj), tb0 = 4 * (blockIdx.y % ngj);
  const int nta = (TA - ta0) < 4 ? (TA - ta0) : 4, ntb = (TB - tb0) < 4 ? (TB - tb0) : 4;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = (r0 + rpb) < N ? (r0 + rpb) : N;
  const int kr = lane / 16, cl = lane % 16;
  d4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
  for (int64_t r = r0 + 4 * wave; r < r1; r += 16) {
    const int64_t row = r + kr;
    const bool rv = row < r1;
    double av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = 16 * (ta0 + i) + cl;
      av[i] = (rv && i < nta && c < a) ? (double)X[row * ldx + c] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 16 * (tb0 + j) + cl;
      bv[j] = (rv && j < ntb && c < b) ? (double)Y[row * ldy + c] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (i < nta && j < ntb)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
  }
  // D layout (FP64 16x16x4): register v of lane l holds row 4 v + l/16, column l % 16
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (i < nta && j < ntb) {
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wave][4 * lane + v] = acc[i][j][v];
        __syncthreads();
        if (wave == 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double s = ((red[0][4 * lane + v] + red[1][4 * lane + v]) + red[2][4 * lane + v]) +
                             red[3][4 * lane + v];
            const int oi = 16 * (ta0 + i) + 4 * v + kr, oj = 16 * (tb0 + j) + cl;
            if (oi < a && oj < b) part[((int64_t)blockIdx.x * a + oi) * b + oj] = s;
          }
        }
      }
    }
}

// X^T X for at most NT = 5 column tiles: the NT (NT + 1) / 2 tiles i <= j in one
// pass over the rows (each row read once; the general kernel above reads it once
// per group of four tiles and computes every tile), the result written to both
// (i, j) and (j, i).  Same fragment layout, row stepping and wave-order sums as
// k_gram; the values of the next 4-row step are loaded before the products of
// the current one.
template <typename T, int NT>
__global__ __launch_bounds__(256) void k_gram_sym(int64_t N, int a, const T *__restrict__ X, int ldx,
                                                  int64_t rpb, double *__restrict__ part) {
  __shared__ double red[4][256];
  constexpr int NP = NT * (NT + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = (r0 + rpb) < N ? (r0 + rpb) : N;
  const int kr = lane / 16, cl = lane % 16;
  d4_t acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = d4_t{0.0, 0.0, 0.0, 0.0};
  auto load = [&](int64_t r, double (&v)[NT]) {
    const int64_t row = r + kr;
    const bool rv = row < r1;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int c = 16 * i + cl;
      v[i] = (rv && c < a) ? (double)X[row * ldx + c] : 0.0;
    }
  };
  double nx[NT];
  int64_t r = r0 + 4 * wave;
  if (r < r1) load(r, nx);
  for (; r < r1; r += 16) {
    double cu[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) cu[i] = nx[i];
    if (r + 16 < r1) load(r + 16, nx);
    int p = 0;
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = i; j < NT; ++j, ++p)
        acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(cu[i], cu[j], acc[p], 0, 0, 0);
  }
  int p = 0;
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = i; j < NT; ++j, ++p) {
      __syncthreads();
#pragma unroll
      for (int v = 0; v < 4; ++v) red[wave][4 * lane + v] = acc[p][v];
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double sv = ((red[0][4 * lane + v] + red[1][4 * lane + v]) + red[2][4 * lane + v]) +
                            red[3][4 * lane + v];
          const int oi = 16 * i + 4 * v + kr, oj = 16 * j + cl;
          if (oi < a && oj < a) {
            part[((int64_t)blockIdx.x * a + oi) * a + oj] = sv;
            part[((int64_t)blockIdx.x * a + oj) * a + oi] = sv;
          }
        }
      }
    }
}

// out[e] = sum over row blocks c (in order) of part[c][e]: 64 elements per
// block, four lanes per element take blocks c = g, g+4, ... then add in order.
__global__ __launch_bounds__(256) void k_gram_reduce(int64_t nchunks, int64_t ab,
                                                     const double *__restrict__ part,
                                                     double *__restrict__ out) {
  __shared__ double sh[4][64];
  const int el = threadIdx.x % 64, g = threadIdx.x / 64;
  const int64_t e = (int64_t)blockIdx.x * 64 + el;
  double s = 0.0;
  if (e < ab) {
#pragma unroll 8
    for (int64_t c = g; c < nchunks; c += 4) s += part[c * ab + e];
  }
  sh[g][el] = s;
  __syncthreads();
  if (g == 0 && e < ab) out[e] = ((sh[0][el] + sh[1][el]) + sh[2][el]) + sh[3][el];
}

template <typename T>
hipError_t launch_gram(int64_t N, int a, const T *X, int ldx, int b, const T *Y, int ldy,
                       double *part, int64_t part_cap, double *out, hipStream_t s) {
  const int64_t ab = (int64_t)a * b;
  if (ab == 0) return hipSuccess;
  const int TA = (a + 15) / 16, TB = (b + 15) / 16;
  if (X == Y && a == b && ldx == ldy && TA <= 5) {
    // X^T X: one pass, upper tiles only; one block per resident slot (two per
    // CU at four or five tiles, whose accumulators leave two waves per SIMD)
    int64_t nx = (N + 63) / 64;
    const int64_t xmax = TA >= 4 ? 512 : 1024;
    if (nx > xmax) nx = xmax;
    if (nx * ab > part_cap) nx = part_cap / ab;
    if (nx < 1) nx = 1;
    if (nx * ab > part_cap) return hipErrorInvalidValue;
    const int64_t rpb = N > 0 ? ((N + nx - 1) / nx + 3) / 4 * 4 : 4;
    nx = N > 0 ? (N + rpb - 1) / rpb : 1;
    switch (TA) {
#define BMG_GRAM_SYM(NTv)                                                                                  \
  hipLaunchKernelGGL((k_gram_sym<T, NTv>), dim3((unsigned)nx), dim3(256), 0, s, N, a, X, ldx, rpb, part)
      case 1: BMG_GRAM_SYM(1); break;
      case 2: BMG_GRAM_SYM(2); break;
      case 3: BMG_GRAM_SYM(3); break;
      case 4: BMG_GRAM_SYM(4); break;
      default: BMG_GRAM_SYM(5); break;
#undef BMG_GRAM_SYM
    }
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((ab + 63) / 64)), dim3(256), 0, s, nx, ab,
                       (const double *)part, out);
    return hipGetLastError();
  }
  const int ny = ((TA + 3) / 4) * ((TB + 3) / 4);
  int64_t nx = (N + 63) / 64;                   // >= 64 rows per block
  const int64_t xmax = (1024 + ny - 1) / ny;    // about 1024 blocks in all
  if (nx > xmax) nx = xmax;
  if (nx * ab > part_cap) nx = part_cap / ab;
  if (nx < 1) nx = 1;
  if (nx * ab > part_cap) return hipErrorInvalidValue;
  const int64_t rpb = N > 0 ? ((N + nx - 1) / nx + 3) / 4 * 4 : 4;
  nx = N > 0 ? (N + rpb - 1) / rpb : 1;
  hipLaunchKernelGGL((k_gram<T>), dim3((unsigned)nx, (unsigned)ny), dim3(256), 0, s, N, a, X, ldx,
                     b, Y, ldy, rpb, part);
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((ab + 63) / 64)), dim3(256), 0, s, nx, ab,
                     (const double *)part, out);
  return hipGetLastError();
}

// ============================================================================ tall x small product
// C[N x b] = X[N x a] M[a x b] + beta C.  64 x 64 output tiles, K-chunks of 16
// staged in LDS, 4 x 4 outputs per thread, FP64 accumulation.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_ts(int64_t N, int a, const T *__restrict__ X,
                                                 int ldx, int b, const double *__restrict__ M,
                                                 int ldm, T *__restrict__ C, int ldc,
                                                 double beta) {
  __shared__ double xs[64][17];
  __shared__ double ms[16][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < a; k0 += 16) {
    for (int t = threadIdx.x; t < 64 * 16; t += 256) {
      const int rr = t / 16, kk = t % 16;
      const int64_t r = r0 + rr;
      xs[rr][kk] = (r < N && k0 + kk < a) ? (double)X[r * ldx + k0 + kk] : 0.0;
      const int mk = t / 64, mc = t % 64;
      ms[mk][mc] = (k0 + mk < a && c0 + mc < b) ? M[(int64_t)(k0 + mk) * ldm + c0 + mc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double xv[4], mv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xv[i] = xs[tr * 4 + i][kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) mv[j] = ms[kk][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += xv[i] * mv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + tr * 4 + i;
    if (r >= N) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tc + 16 * j;
      if (c >= b) continue;
      double v = acc[i][j];
      if (beta != 0.0) v += beta * (double)C[r * ldc + c];
      C[r * ldc + c] = (T)v;
    }
  }
}

// The same product with 64 x (16 NC) output tiles (4 x NC outputs per
// thread): for b in (64, 16 NC] one tile spans all of M's columns, so X is
// read once instead of once per 64 columns.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_gemm_ts_w(int64_t N, int a, const T *__restrict__ X, int ldx,
                                                   int b, const double *__restrict__ M, int ldm,
                                                   T *__restrict__ C, int ldc, double beta) {
  __shared__ double xs[64][17];
  __shared__ double ms[16][16 * NC + 1];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  double acc[4][NC] = {};
  for (int k0 = 0; k0 < a; k0 += 16) {
    for (int t = threadIdx.x; t < 64 * 16; t += 256) {
      const int rr = t / 16, kk = t % 16;
      const int64_t r = r0 + rr;
      xs[rr][kk] = (r < N && k0 + kk < a) ? (double)X[r * ldx + k0 + kk] : 0.0;
    }
    for (int t = threadIdx.x; t < 16 * 16 * NC; t += 256) {
      const int mk = t / (16 * NC), mc = t % (16 * NC);
      ms[mk][mc] = (k0 + mk < a && mc < b) ? M[(int64_t)(k0 + mk) * ldm + mc] : 0.0;
    }
    __syncthreads();
    // the last chunk holds a % 16 terms: the rest (zeros) are skipped
    const int kn = (a - k0) < 16 ? (a - k0) : 16;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      if (kk >= kn) break;
      double xv[4], mv[NC];
#pragma unroll
      for (int i = 0; i < 4; ++i) xv[i] = xs[tr * 4 + i][kk];
#pragma unroll
      for (int j = 0; j < NC; ++j) mv[j] = ms[kk][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[i][j] += xv[i] * mv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + tr * 4 + i;
    if (r >= N) continue;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c = tc + 16 * j;
      if (c >= b) continue;
      double v = acc[i][j];
      if (beta != 0.0) v += beta * (double)C[r * ldc + c];
      C[r * ldc + c] = (T)v;
    }
  }
}

// The same product with 32 x 32 output tiles (K-chunks of 32, 2 x 2 outputs
// per thread): four times the blocks, for products too short to fill the
// chip with 64 x 64 tiles.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_ts32(int64_t N, int a, const T *__restrict__ X,
                                                   int ldx, int b, const double *__restrict__ M,
                                                   int ldm, T *__restrict__ C, int ldc,
                                                   double beta) {
  __shared__ double xs[32][33];
  __shared__ double ms[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 32;
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  double acc[2][2] = {};
  for (int k0 = 0; k0 < a; k0 += 32) {
    for (int t = threadIdx.x; t < 32 * 32; t += 256) {
      const int rr = t / 32, kk = t % 32;
      const int64_t r = r0 + rr;
      xs[rr][kk] = (r < N && k0 + kk < a) ? (double)X[r * ldx + k0 + kk] : 0.0;
      const int mk = t / 32, mc = t % 32;
      ms[mk][mc] = (k0 + mk < a && c0 + mc < b) ? M[(int64_t)(k0 + mk) * ldm + c0 + mc] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) {
      const double x0 = xs[tr * 2][kk], x1 = xs[tr * 2 + 1][kk];
      const double m0 = ms[kk][tc], m1 = ms[kk][tc + 16];
      acc[0][0] += x0 * m0;
      acc[0][1] += x0 * m1;
      acc[1][0] += x1 * m0;
      acc[1][1] += x1 * m1;
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int64_t r = r0 + tr * 2 + i;
    if (r >= N) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = c0 + tc + 16 * j;
      if (c >= b) continue;
      double v = acc[i][j];
      if (beta != 0.0) v += beta * (double)C[r * ldc + c];
      C[r * ldc + c] = (T)v;
    }
  }
}

template <typename T>
hipError_t launch_gemm_ts(int64_t N, int a, const T *X, int ldx, int b, const double *M, int ldm,
                          T *C, int ldc, double beta, hipStream_t s) {
  if (N == 0 || b == 0) return hipSuccess;
  if (a == 0) {  // C = beta C
    if (beta == 1.0) return hipSuccess;
    return launch_axpy<T>(N, b, beta - 1.0, C, ldc, C, ldc, s);
  }
  const int64_t tiles64 = ((N + 63) / 64) * ((b + 63) / 64);
  if (tiles64 >= 1024 && b > 64 && b <= 128) {
    const dim3 grid((unsigned)((N + 63) / 64));
    if (b <= 80)
      hipLaunchKernelGGL((k_gemm_ts_w<T, 5>), grid, dim3(256), 0, s, N, a, X, ldx, b, M, ldm, C, ldc, beta);
    else if (b <= 96)
      hipLaunchKernelGGL((k_gemm_ts_w<T, 6>), grid, dim3(256), 0, s, N, a, X, ldx, b, M, ldm, C, ldc, beta);
    else
      hipLaunchKernelGGL((k_gemm_ts_w<T, 8>), grid, dim3(256), 0, s, N, a, X, ldx, b, M, ldm, C, ldc, beta);
    return hipGetLastError();
  }
  if (tiles64 < 1024) {
    dim3 grid((unsigned)((N + 31) / 32), (unsigned)((b + 31) / 32));
    hipLaunchKernelGGL((k_gemm_ts32<T>), grid, dim3(256), 0, s, N, a, X, ldx, b, M, ldm, C, ldc,
                       beta);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((b + 63) / 64));
  hipLaunchKernelGGL((k_gemm_ts<T>), grid, dim3(256), 0, s, N, a, X, ldx, b, M, ldm, C, ldc, beta);
  return hipGetLastError();
}

// ============================================================================ elementwise
template <typename T>
__global__ void k_fill(T *p, int64_t rows, int cols, int ld, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int64_t r = i / cols;
  const int c = (int)(i % cols);
  p[r * ld + c] = (T)v;
}
template <typename T>
hipError_t launch_fill(T *p, int64_t rows, int cols, int ld, double v, hipStream_t s) {
  const int64_t n = rows * cols;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, rows, cols,
                     ld, v);
  return hipGetLastError();
}

template <typename T>
__global__ void k_axpy(int64_t rows, int cols, double a, const T *X, int ldx, T *Y, int ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int64_t r = i / cols;
  const int c = (int)(i % cols);
  Y[r * ldy + c] = (T)((double)Y[r * ldy + c] + a * (double)X[r * ldx + c]);
}
template <typename T>
hipError_t launch_axpy(int64_t rows, int cols, double a, const T *X, int ldx, T *Y, int ldy,
                       hipStream_t s) {
  const int64_t n = rows * cols;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_axpy<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rows, cols, a,
                     X, ldx, Y, ldy);
  return hipGetLastError();
}

template <typename T>
__global__ void k_copy_cols(int64_t rows, int cols, const T *X, int ldx, T *Y, int ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int64_t r = i / cols;
  const int c = (int)(i % cols);
  Y[r * ldy + c] = X[r * ldx + c];
}
template <typename T>
hipError_t launch_copy_cols(int64_t rows, int cols, const T *X, int ldx, T *Y, int ldy,
                            hipStream_t s) {
  const int64_t n = rows * cols;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_copy_cols<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rows,
                     cols, X, ldx, Y, ldy);
  return hipGetLastError();
}

template <typename Tin, typename Tout>
__global__ void k_convert(int64_t n, const Tin *x, Tout *y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (Tout)x[i];
}
template <typename Tin, typename Tout>
hipError_t launch_convert(int64_t n, const Tin *x, Tout *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                     x, y);
  return hipGetLastError();
}

template <typename Tin, typename Tout>
__global__ void k_convert_cols(int64_t rows, int cols, const Tin *X, int ldx, Tout *Y, int ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int64_t r = i / cols;
  const int c = (int)(i % cols);
  Y[r * ldy + c] = cvt<Tout, Tin>(X[r * ldx + c]);
}
template <typename Tin, typename Tout>
hipError_t launch_convert_cols(int64_t rows, int cols, const Tin *X, int ldx, Tout *Y, int ldy,
                               hipStream_t s) {
  const int64_t n = rows * cols;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert_cols<Tin, Tout>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     rows, cols, X, ldx, Y, ldy);
  return hipGetLastError();
}
template hipError_t launch_convert_cols<double, float>(int64_t, int, const double *, int, float *, int,
                                                       hipStream_t);
template hipError_t launch_convert_cols<float, double>(int64_t, int, const float *, int, double *, int,
                                                       hipStream_t);
template hipError_t launch_convert_cols<float, bf16_t>(int64_t, int, const float *, int, bf16_t *, int,
                                                       hipStream_t);
template hipError_t launch_convert_cols<double, double>(int64_t, int, const double *, int, double *,
                                                        int, hipStream_t);

// ============================================================================ counter-based normals
// SplitMix64 (Steele, Lea, Flood 2014): draw c of stream (seed, id) is
// mix64(x0 + (c+1) * gamma) with x0 = seed ^ (id * 0xD1B54A32D192ED03);
// uniform ((v >> 11) + 0.5) 2^-53; normal i = Box-Muller on draws 2i, 2i+1.
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
template <typename T>
__global__ void k_normals(uint64_t seed, uint64_t stream, int64_t rows, int cols, int ld, T *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const uint64_t x0 = seed ^ (stream * 0xD1B54A32D192ED03ULL);
  const uint64_t g = 0x9E3779B97F4A7C15ULL;
  const uint64_t v1 = mix64(x0 + (uint64_t)(2 * i + 1) * g);
  const uint64_t v2 = mix64(x0 + (uint64_t)(2 * i + 2) * g);
  const double u1 = ((double)(v1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((double)(v2 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  out[(i / cols) * ld + (i % cols)] = (T)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}
template <typename T>
hipError_t launch_normals(uint64_t seed, uint64_t stream, int64_t rows, int cols, int ld, T *out,
                          hipStream_t s) {
  const int64_t count = rows * cols;
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL((k_normals<T>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, seed,
                     stream, rows, cols, ld, out);
  return hipGetLastError();
}

__global__ void k_gather_perm(int64_t nnz, const int32_t *perm, const double *in, double *out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nnz) out[q] = in[perm[q]];
}
hipError_t launch_gather_perm(int64_t nnz, const int32_t *perm, const double *in, double *out,
                              hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_perm, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, perm,
                     in, out);
  return hipGetLastError();
}

// ============================================================================ setup kernels
__global__ void k_row_ids(int64_t m, const int64_t *row_ptr, int32_t *rid) {
  // one thread per entry, binary search over row_ptr
  const int64_t nnz = row_ptr[m];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = m;  // find i with row_ptr[i] <= p < row_ptr[i+1]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (row_ptr[mid] <= p) lo = mid; else hi = mid;
    }
    rid[p] = (int32_t)lo;
  }
}
hipError_t launch_row_ids(int64_t m, const int64_t *row_ptr, int32_t *rid, hipStream_t s) {
  hipLaunchKernelGGL(k_row_ids, dim3(4096), dim3(256), 0, s, m, row_ptr, rid);
  return hipGetLastError();
}

__global__ void k_iota(int64_t n, int32_t *p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}
hipError_t launch_iota(int64_t n, int32_t *p, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, p);
  return hipGetLastError();
}

__global__ void k_gather_csc(int64_t nnz, const int32_t *perm, const int32_t *rid,
                             const double *val, int32_t *crow, double *cval) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  const int32_t p = perm[q];
  crow[q] = rid[p];
  cval[q] = val[p];
}
hipError_t launch_gather_csc(int64_t nnz, const int32_t *perm, const int32_t *rid,
                             const double *val, int32_t *crow, double *cval, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_csc, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, perm,
                     rid, val, crow, cval);
  return hipGetLastError();
}

// cptr[j] = first position whose sorted column is >= j  (cptr[n] = nnz)
__global__ void k_col_ptr(int64_t nnz, int64_t n, const int32_t *sc, int64_t *cptr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const int64_t cur = sc[p];
  const int64_t prev = p == 0 ? -1 : (int64_t)sc[p - 1];
  for (int64_t j = prev + 1; j <= cur; ++j) cptr[j] = p;
  if (p == nnz - 1)
    for (int64_t j = cur + 1; j <= n; ++j) cptr[j] = nnz;
}
hipError_t launch_col_ptr(int64_t nnz, int64_t n, const int32_t *sorted_col, int64_t *cptr,
                          hipStream_t s) {
  if (nnz == 0) return launch_fill<int64_t>(cptr, n + 1, 1, 1, 0.0, s);
  hipLaunchKernelGGL(k_col_ptr, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, n,
                     sorted_col, cptr);
  return hipGetLastError();
}

// flags: bit 0 unsorted or duplicate column, bit 1 column out of range,
// bit 2 non-finite value, bit 3 row_ptr not non-decreasing.
__global__ void k_check_csr(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
                            const double *val, const int32_t *rid, int *flags) {
  const int64_t nnz = row_ptr[m];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    int f = 0;
    const int32_t c = col[p];
    if (c < 0 || c >= n) f |= 2;
    if (!isfinite(val[p])) f |= 4;
    if (p > row_ptr[rid[p]] && col[p - 1] >= c) f |= 1;
    if (f) atomicOr(flags, f);
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    if (row_ptr[i + 1] < row_ptr[i]) atomicOr(flags, 8);
}
hipError_t launch_check_csr(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
                            const double *val, const int32_t *rid, int *flags, hipStream_t s) {
  hipLaunchKernelGGL(k_check_csr, dim3(2048), dim3(256), 0, s, m, n, row_ptr, col, val, rid, flags);
  return hipGetLastError();
}

// ============================================================================ instantiations
#define BMG_INST(T)                                                                              \
  template hipError_t launch_gram<T>(int64_t, int, const T *, int, int, const T *, int, double *,  \
                                     int64_t, double *, hipStream_t);                              \
  template hipError_t launch_gemm_ts<T>(int64_t, int, const T *, int, int, const double *, int,   \
                                        T *, int, double, hipStream_t);                            \
  template hipError_t launch_fill<T>(T *, int64_t, int, int, double, hipStream_t);                \
  template hipError_t launch_axpy<T>(int64_t, int, double, const T *, int, T *, int, hipStream_t); \
  template hipError_t launch_copy_cols<T>(int64_t, int, const T *, int, T *, int, hipStream_t);  \
  template hipError_t launch_normals<T>(uint64_t, uint64_t, int64_t, int, int, T *, hipStream_t);
BMG_INST(double)
BMG_INST(float)
template hipError_t launch_fill<int64_t>(int64_t *, int64_t, int, int, double, hipStream_t);
template hipError_t launch_convert<double, float>(int64_t, const double *, float *, hipStream_t);
template hipError_t launch_convert<float, double>(int64_t, const float *, double *, hipStream_t);

}  // namespace bmg
