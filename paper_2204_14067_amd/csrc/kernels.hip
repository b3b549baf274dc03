// HIP kernels for gfx950 (CDNA4, wave64) of the BM-Global matrix-completion
// hot path.
//
// Sparse passes over Omega are memory-bound (the paper's own observation on
// the subspace products, Suppl. A.1.6): per stored entry they stream a 4-byte
// index and one value and gather one row of a dense factor.  Layout choice:
// a group of G lanes owns one row of Omega; each lane holds a 16-byte slice
// (2 doubles / 4 floats) of the k-vectors, so one gathered factor row is a
// single fully-used cache-line access, dot products need log2(G) butterfly
// steps inside the group, and the accumulated output row never leaves
// registers until the row ends.  Index/value streams are read with
// non-temporal loads so they do not evict the gathered factor rows from L2.
//
// Determinism: no floating-point atomics anywhere.  Scalar sums are written
// per wave and added in a fixed order by a one-block kernel; long rows are
// split into fixed pieces whose partial rows are added in piece order.
#include <hip/hip_runtime.h>

#include "bmg_internal.h"

namespace bmg {

template <typename T> struct VT;
template <> struct VT<double> { static constexpr int V = 2; };
template <> struct VT<float> { static constexpr int V = 4; };

template <typename T>
__device__ __forceinline__ T nt_load(const T *p) { return __builtin_nontemporal_load(p); }

// Load V consecutive elements row[f0 .. f0+V) with per-element bound lim
// (elements at or beyond lim read as 0 and are never touched).
template <typename T, int V>
__device__ __forceinline__ void ldv(const T *__restrict__ row, int f0, int lim, T (&x)[V]) {
  if (f0 + V <= lim) {
    if constexpr (sizeof(T) == 8) {
      const double2 v = *reinterpret_cast<const double2 *>(row + f0);
      x[0] = v.x; x[1] = v.y;
    } else {
      const float4 v = *reinterpret_cast<const float4 *>(row + f0);
      x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e) x[e] = (f0 + e < lim) ? row[f0 + e] : T(0);
  }
}

template <typename T, int V>
__device__ __forceinline__ void stv(T *__restrict__ row, int f0, int lim, const T (&x)[V]) {
  if (f0 + V <= lim) {
    if constexpr (sizeof(T) == 8) {
      *reinterpret_cast<double2 *>(row + f0) = make_double2(x[0], x[1]);
    } else {
      *reinterpret_cast<float4 *>(row + f0) = make_float4(x[0], x[1], x[2], x[3]);
    }
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e)
      if (f0 + e < lim) row[f0 + e] = x[e];
  }
}

// Butterfly sum inside a lane group of G (xor offsets 1 .. G/2).
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Sum across the 64/G groups of a wave (xor offsets G .. 32).
template <int G, typename T>
__device__ __forceinline__ T slot_sum(T v) {
#pragma unroll
  for (int o = G; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

constexpr int UNROLL = 4;
constexpr int WAVES_PER_BLOCK = 4;

__host__ __device__ inline int64_t short_waves(const Plan &pl, int G) {
  const int S = 64 / G;
  return (pl.n_short + S - 1) / S;
}

// ============================================================================ fused residual + product
// For one entry range [p, p + n*step) of a row: r = x.y_j - a_p ; acc += r y_j ; ss += r^2.
template <typename T, int G, int V>
__device__ __forceinline__ void grad_block(const Plan &pl, const T *__restrict__ a,
                                           const T *__restrict__ Y, int ldy, int k, int f0,
                                           const T (&x)[V], T (&acc)[V], double &ss, bool leader,
                                           int64_t p, int64_t step, int n) {
  int j[UNROLL];
  T av[UNROLL];
  T y[UNROLL][V];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    if (u < n) {
      j[u] = nt_load(pl.idx + p + u * step);
      av[u] = nt_load(a + p + u * step);
    } else {
      j[u] = -1;
      av[u] = T(0);
    }
  }
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    if (j[u] >= 0) ldv<T, V>(Y + (int64_t)j[u] * ldy, f0, k, y[u]);
    else {
#pragma unroll
      for (int e = 0; e < V; ++e) y[u][e] = T(0);
    }
  }
  T d[UNROLL];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    T s = T(0);
#pragma unroll
    for (int e = 0; e < V; ++e) s += x[e] * y[u][e];
    d[u] = s;
  }
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) d[u] = group_sum<G>(d[u]);
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    if (u < n) {
      const T r = d[u] - av[u];
#pragma unroll
      for (int e = 0; e < V; ++e) acc[e] += r * y[u][e];
      if (leader) ss += (double)r * (double)r;
    }
  }
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_grad(Plan pl, const T *__restrict__ a,
                                              const T *__restrict__ X, int ldx,
                                              const T *__restrict__ Y, int ldy, int k, double lam,
                                              T *__restrict__ Out, int ldo,
                                              T *__restrict__ partial, double *__restrict__ wsum,
                                              int64_t total_waves) {
  constexpr int V = VT<T>::V, S = 64 / G, WB = G * V;
  const int lane = threadIdx.x & 63, slot = lane / G, sub = lane % G, f0 = sub * V;
  const int64_t gw = (int64_t)blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
  const int64_t sw = short_waves(pl, G);
  const bool leader = (sub == 0);
  double ss = 0.0;
  T acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = T(0);
  if (gw < sw) {
    const int64_t ri = gw * S + slot;
    if (ri < pl.n_short) {
      const int row = pl.short_rows[ri];
      T x[V];
      ldv<T, V>(X + (int64_t)row * ldx, f0, k, x);
      const int64_t beg = pl.ptr[row], end = pl.ptr[row + 1];
      for (int64_t p = beg; p < end; p += UNROLL) {
        const int n = (int)((end - p) < UNROLL ? (end - p) : UNROLL);
        grad_block<T, G, V>(pl, a, Y, ldy, k, f0, x, acc, ss, leader, p, 1, n);
      }
#pragma unroll
      for (int e = 0; e < V; ++e) acc[e] += (T)lam * x[e];
      stv<T, V>(Out + (int64_t)row * ldo, f0, k, acc);
    }
  } else if (gw < total_waves) {
    const int64_t pc = gw - sw;
    const int row = pl.piece_row[pc];
    const int64_t beg = pl.piece_beg[pc];
    int64_t end = pl.ptr[row + 1];
    if (end > beg + pl.chunk) end = beg + pl.chunk;
    T x[V];
    ldv<T, V>(X + (int64_t)row * ldx, f0, k, x);
    for (int64_t p = beg + slot; p < end; p += (int64_t)S * UNROLL) {
      const int64_t rem = (end - p + S - 1) / S;
      const int n = (int)(rem < UNROLL ? rem : UNROLL);
      grad_block<T, G, V>(pl, a, Y, ldy, k, f0, x, acc, ss, leader, p, S, n);
    }
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] = slot_sum<G>(acc[e]);
    if (slot == 0) stv<T, V>(partial + pc * WB, f0, WB, acc);
  }
  ss = wave_sum(ss);
  if (lane == 0 && gw < total_waves) wsum[gw] = ss;
}

// Long rows: Out_row = sum of piece partials (piece order) + lam * x_row.
template <typename T, int G>
__global__ __launch_bounds__(256) void k_grad_fix(Plan pl, const T *__restrict__ partial,
                                                  const T *__restrict__ X, int ldx, int k,
                                                  double lam, T *__restrict__ Out, int ldo) {
  constexpr int V = VT<T>::V, WB = G * V;
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int f0 = (threadIdx.x % G) * V;
  if (g >= pl.n_long) return;
  const int row = pl.long_rows[g];
  T acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = T(0);
  for (int pc = pl.long_p0[g]; pc < pl.long_p0[g + 1]; ++pc) {
    T t[V];
    ldv<T, V>(partial + (int64_t)pc * WB, f0, WB, t);
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] += t[e];
  }
  T x[V];
  ldv<T, V>(X + (int64_t)row * ldx, f0, k, x);
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] += (T)lam * x[e];
  stv<T, V>(Out + (int64_t)row * ldo, f0, k, acc);
}

// ============================================================================ sampled residual
template <typename T, int G, int V>
__device__ __forceinline__ void sddmm_block(const Plan &pl, const T *__restrict__ a,
                                            const T *__restrict__ Y, int ldy, int k, int f0,
                                            const T (&x)[V], T *__restrict__ R, double &ss,
                                            double &sx, bool leader, int64_t p, int64_t step,
                                            int n) {
  int j[UNROLL];
  T av[UNROLL];
  T y[UNROLL][V];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    if (u < n) {
      j[u] = nt_load(pl.idx + p + u * step);
      av[u] = a ? nt_load(a + p + u * step) : T(0);
    } else {
      j[u] = -1;
      av[u] = T(0);
    }
  }
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    if (j[u] >= 0) ldv<T, V>(Y + (int64_t)j[u] * ldy, f0, k, y[u]);
    else {
#pragma unroll
      for (int e = 0; e < V; ++e) y[u][e] = T(0);
    }
  }
  T d[UNROLL];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    T s = T(0);
#pragma unroll
    for (int e = 0; e < V; ++e) s += x[e] * y[u][e];
    d[u] = group_sum<G>(s);
  }
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    if (u < n && leader) {
      const T r = d[u] - av[u];
      if (R) R[p + u * step] = r;
      ss += (double)r * (double)r;
      sx += (double)r * (double)d[u];
    }
  }
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_sddmm(Plan pl, const T *__restrict__ a,
                                               const T *__restrict__ X, int ldx,
                                               const T *__restrict__ Y, int ldy, int k,
                                               T *__restrict__ R, double *__restrict__ wsum,
                                               int64_t total_waves) {
  constexpr int V = VT<T>::V, S = 64 / G;
  const int lane = threadIdx.x & 63, slot = lane / G, sub = lane % G, f0 = sub * V;
  const int64_t gw = (int64_t)blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
  const int64_t sw = short_waves(pl, G);
  const bool leader = (sub == 0);
  double ss = 0.0, sx = 0.0;
  if (gw < sw) {
    const int64_t ri = gw * S + slot;
    if (ri < pl.n_short) {
      const int row = pl.short_rows[ri];
      T x[V];
      ldv<T, V>(X + (int64_t)row * ldx, f0, k, x);
      const int64_t beg = pl.ptr[row], end = pl.ptr[row + 1];
      for (int64_t p = beg; p < end; p += UNROLL) {
        const int n = (int)((end - p) < UNROLL ? (end - p) : UNROLL);
        sddmm_block<T, G, V>(pl, a, Y, ldy, k, f0, x, R, ss, sx, leader, p, 1, n);
      }
    }
  } else if (gw < total_waves) {
    const int64_t pc = gw - sw;
    const int row = pl.piece_row[pc];
    const int64_t beg = pl.piece_beg[pc];
    int64_t end = pl.ptr[row + 1];
    if (end > beg + pl.chunk) end = beg + pl.chunk;
    T x[V];
    ldv<T, V>(X + (int64_t)row * ldx, f0, k, x);
    for (int64_t p = beg + slot; p < end; p += (int64_t)S * UNROLL) {
      const int64_t rem = (end - p + S - 1) / S;
      const int n = (int)(rem < UNROLL ? rem : UNROLL);
      sddmm_block<T, G, V>(pl, a, Y, ldy, k, f0, x, R, ss, sx, leader, p, S, n);
    }
  }
  ss = wave_sum(ss);
  sx = wave_sum(sx);
  if (lane == 0 && gw < total_waves) {
    wsum[2 * gw] = ss;
    wsum[2 * gw + 1] = sx;
  }
}

// ============================================================================ sparse x dense
template <typename T, int G, int V>
__device__ __forceinline__ void spmm_block(const Plan &pl, const T *__restrict__ Sv,
                                           const T *__restrict__ B, int ldb, int wq, int f0,
                                           T (&acc)[V], int64_t p, int64_t step, int n) {
  int j[UNROLL];
  T sv[UNROLL];
  T b[UNROLL][V];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    if (u < n) {
      j[u] = nt_load(pl.idx + p + u * step);
      sv[u] = nt_load(Sv + p + u * step);
    } else {
      j[u] = -1;
      sv[u] = T(0);
    }
  }
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    if (j[u] >= 0) ldv<T, V>(B + (int64_t)j[u] * ldb, f0, wq, b[u]);
    else {
#pragma unroll
      for (int e = 0; e < V; ++e) b[u][e] = T(0);
    }
  }
#pragma unroll
  for (int u = 0; u < UNROLL; ++u)
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] += sv[u] * b[u][e];
}

// out = coef * acc + x_row . M[:, slice]
template <typename T, int V>
__device__ __forceinline__ void lowrank_epilogue(T (&acc)[V], double coef, const T *__restrict__ xr,
                                                 int kx, const T *__restrict__ M, int ldm, int wq,
                                                 int f0) {
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] *= (T)coef;
  for (int r = 0; r < kx; ++r) {
    const T xv = xr[r];
    T mv[V];
    ldv<T, V>(M + (int64_t)r * ldm, f0, wq, mv);
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] += xv * mv[e];
  }
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_spmm(Plan pl, const T *__restrict__ Sv,
                                              const T *__restrict__ B, int ldb, int wq,
                                              double coef, const T *__restrict__ X, int ldx,
                                              int kx, const T *__restrict__ M, int ldm,
                                              T *__restrict__ C, int ldc,
                                              T *__restrict__ partial, int64_t total_waves) {
  constexpr int V = VT<T>::V, S = 64 / G, WB = G * V;
  const int lane = threadIdx.x & 63, slot = lane / G, sub = lane % G, f0 = sub * V;
  const int64_t gw = (int64_t)blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
  const int64_t sw = short_waves(pl, G);
  T acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = T(0);
  if (gw < sw) {
    const int64_t ri = gw * S + slot;
    if (ri < pl.n_short) {
      const int row = pl.short_rows[ri];
      const int64_t beg = pl.ptr[row], end = pl.ptr[row + 1];
      for (int64_t p = beg; p < end; p += UNROLL) {
        const int n = (int)((end - p) < UNROLL ? (end - p) : UNROLL);
        spmm_block<T, G, V>(pl, Sv, B, ldb, wq, f0, acc, p, 1, n);
      }
      lowrank_epilogue<T, V>(acc, coef, X + (int64_t)row * ldx, kx, M, ldm, wq, f0);
      stv<T, V>(C + (int64_t)row * ldc, f0, wq, acc);
    }
  } else if (gw < total_waves) {
    const int64_t pc = gw - sw;
    const int row = pl.piece_row[pc];
    const int64_t beg = pl.piece_beg[pc];
    int64_t end = pl.ptr[row + 1];
    if (end > beg + pl.chunk) end = beg + pl.chunk;
    for (int64_t p = beg + slot; p < end; p += (int64_t)S * UNROLL) {
      const int64_t rem = (end - p + S - 1) / S;
      const int n = (int)(rem < UNROLL ? rem : UNROLL);
      spmm_block<T, G, V>(pl, Sv, B, ldb, wq, f0, acc, p, S, n);
    }
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] = slot_sum<G>(acc[e]);
    if (slot == 0) stv<T, V>(partial + pc * WB, f0, WB, acc);
  }
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_spmm_fix(Plan pl, const T *__restrict__ partial,
                                                  double coef, const T *__restrict__ X, int ldx,
                                                  int kx, const T *__restrict__ M, int ldm, int wq,
                                                  T *__restrict__ C, int ldc) {
  constexpr int V = VT<T>::V, WB = G * V;
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int f0 = (threadIdx.x % G) * V;
  if (g >= pl.n_long) return;
  const int row = pl.long_rows[g];
  T acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = T(0);
  for (int pc = pl.long_p0[g]; pc < pl.long_p0[g + 1]; ++pc) {
    T t[V];
    ldv<T, V>(partial + (int64_t)pc * WB, f0, WB, t);
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] += t[e];
  }
  lowrank_epilogue<T, V>(acc, coef, X + (int64_t)row * ldx, kx, M, ldm, wq, f0);
  stv<T, V>(C + (int64_t)row * ldc, f0, wq, acc);
}

// ============================================================================ launchers
static inline int pick_G(int width, int V) {
  int need = (width + V - 1) / V;
  int G = 4;
  while (G < need && G < 64) G <<= 1;
  return G;
}

static inline int64_t total_waves(const Plan &pl, int G) { return short_waves(pl, G) + pl.n_pieces; }

static inline dim3 wave_grid(int64_t waves) {
  int64_t b = (waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  return dim3((unsigned)(b > 0 ? b : 1));
}

#define BMG_DISPATCH_G(G, ...)                                   \
  switch (G) {                                                   \
    case 4: { constexpr int GG = 4; __VA_ARGS__; } break;        \
    case 8: { constexpr int GG = 8; __VA_ARGS__; } break;        \
    case 16: { constexpr int GG = 16; __VA_ARGS__; } break;      \
    case 32: { constexpr int GG = 32; __VA_ARGS__; } break;      \
    default: { constexpr int GG = 64; __VA_ARGS__; } break;      \
  }

template <typename T>
hipError_t launch_grad(const Plan &pl, const T *a, const T *X, int ldx, const T *Y, int ldy, int k,
                       double lam, T *Out, int ldo, PassScratch sc, int64_t *waves_out,
                       hipStream_t s) {
  constexpr int V = VT<T>::V;
  if (k > max_width<T>()) return hipErrorInvalidValue;
  const int G = pick_G(k, V);
  const int64_t tw = total_waves(pl, G);
  if (waves_out) *waves_out = tw;
  BMG_DISPATCH_G(G, {
    if (sc.ev0) (void)hipEventRecord(sc.ev0, s);
    hipLaunchKernelGGL((k_grad<T, GG>), wave_grid(tw), dim3(256), 0, s, pl, a, X, ldx, Y, ldy, k,
                       lam, Out, ldo, (T *)sc.partial, sc.wsum, tw);
    if (sc.ev1) (void)hipEventRecord(sc.ev1, s);
    if (pl.n_long > 0) {
      const int64_t thr = pl.n_long * GG;
      hipLaunchKernelGGL((k_grad_fix<T, GG>), dim3((unsigned)((thr + 255) / 256)), dim3(256), 0, s,
                         pl, (const T *)sc.partial, X, ldx, k, lam, Out, ldo);
    }
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_wsum(sc.wsum, tw, 1, sc.result, s);
}

template <typename T>
hipError_t launch_sddmm(const Plan &pl, const T *a, const T *X, int ldx, const T *Y, int ldy, int k,
                        T *R, PassScratch sc, hipStream_t s) {
  constexpr int V = VT<T>::V;
  if (k > max_width<T>()) return hipErrorInvalidValue;
  const int G = pick_G(k, V);
  const int64_t tw = total_waves(pl, G);
  BMG_DISPATCH_G(G, {
    if (sc.ev0) (void)hipEventRecord(sc.ev0, s);
    hipLaunchKernelGGL((k_sddmm<T, GG>), wave_grid(tw), dim3(256), 0, s, pl, a, X, ldx, Y, ldy, k,
                       R, sc.wsum, tw);
    if (sc.ev1) (void)hipEventRecord(sc.ev1, s);
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_wsum(sc.wsum, tw, 2, sc.result, s);
}

template <typename T>
hipError_t launch_spmm(const Plan &pl, const T *Sv, const T *B, int ldb, int q, double coef,
                       const T *X, int ldx, int kx, const T *M, int ldm, T *C, int ldc,
                       PassScratch sc, hipStream_t s) {
  constexpr int V = VT<T>::V;
  const int WMAX = max_width<T>();
  for (int c0 = 0; c0 < q; c0 += WMAX) {
    const int wq = (q - c0) < WMAX ? (q - c0) : WMAX;
    const int G = pick_G(wq, V);
    const int64_t tw = total_waves(pl, G);
    BMG_DISPATCH_G(G, {
      if (sc.ev0 && c0 == 0) (void)hipEventRecord(sc.ev0, s);
      hipLaunchKernelGGL((k_spmm<T, GG>), wave_grid(tw), dim3(256), 0, s, pl, Sv, B + c0, ldb, wq,
                         coef, X, ldx, kx, M ? M + c0 : M, ldm, C + c0, ldc, (T *)sc.partial, tw);
      if (sc.ev1 && c0 + WMAX >= q) (void)hipEventRecord(sc.ev1, s);
      if (pl.n_long > 0) {
        const int64_t thr = pl.n_long * GG;
        hipLaunchKernelGGL((k_spmm_fix<T, GG>), dim3((unsigned)((thr + 255) / 256)), dim3(256), 0,
                           s, pl, (const T *)sc.partial, coef, X, ldx, kx, M ? M + c0 : M, ldm, wq,
                           C + c0, ldc);
      }
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ============================================================================ scalar reduction
// Sums nsum interleaved per-wave partials in a fixed order: thread t adds
// waves t, t+256, ... in increasing order, then a fixed binary tree.
__global__ __launch_bounds__(256) void k_reduce_wsum(const double *__restrict__ wsum, int64_t waves,
                                                     int nsum, double *__restrict__ out) {
  __shared__ double sh[256];
  for (int c = 0; c < nsum; ++c) {
    double s = 0.0;
    for (int64_t w = threadIdx.x; w < waves; w += 256) s += wsum[w * nsum + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
    __syncthreads();
  }
}

hipError_t launch_reduce_wsum(const double *wsum, int64_t waves, int nsum, double *out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_wsum, dim3(1), dim3(256), 0, s, wsum, waves, nsum, out);
  return hipGetLastError();
}

// ============================================================================ tall-skinny Gram
// part[chunk][a][b] = sum over the chunk's rows of X[r, :a]^T Y[r, :b]; then
// out = sum over chunks in chunk order.  64-row x 32-column LDS tiles, FP64.
constexpr int GR_ROWS = 64, GR_T = 32;

template <typename T>
__global__ __launch_bounds__(256) void k_gram(int64_t N, int a, const T *__restrict__ X, int ldx,
                                              int b, const T *__restrict__ Y, int ldy,
                                              int64_t rows_per_chunk, double *__restrict__ part) {
  __shared__ double xs[GR_ROWS][GR_T + 1];
  __shared__ double ys[GR_ROWS][GR_T + 1];
  const int ta = blockIdx.x, tb = blockIdx.y;
  const int64_t chunk = blockIdx.z;
  const int tx = threadIdx.x % GR_T, ty = threadIdx.x / GR_T;  // ty in 0..7
  const int64_t r_beg = chunk * rows_per_chunk;
  int64_t r_end = r_beg + rows_per_chunk;
  if (r_end > N) r_end = N;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r0 = r_beg; r0 < r_end; r0 += GR_ROWS) {
    for (int t = threadIdx.x; t < GR_ROWS * GR_T; t += 256) {
      const int rr = t / GR_T, cc = t % GR_T;
      const int64_t r = r0 + rr;
      const int ca = ta * GR_T + cc, cb = tb * GR_T + cc;
      xs[rr][cc] = (r < r_end && ca < a) ? (double)X[r * ldx + ca] : 0.0;
      ys[rr][cc] = (r < r_end && cb < b) ? (double)Y[r * ldy + cb] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < GR_ROWS; ++rr) {
      const double yv = ys[rr][tx];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] += xs[rr][ty + 8 * i] * yv;
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int ia = ta * GR_T + ty + 8 * i, ib = tb * GR_T + tx;
    if (ia < a && ib < b) part[(chunk * a + ia) * b + ib] = acc[i];
  }
}

__global__ void k_gram_reduce(int64_t nchunks, int64_t ab, const double *__restrict__ part,
                              double *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ab) return;
  double s = 0.0;
  for (int64_t c = 0; c < nchunks; ++c) s += part[c * ab + e];
  out[e] = s;
}

template <typename T>
hipError_t launch_gram(int64_t N, int a, const T *X, int ldx, int b, const T *Y, int ldy,
                       double *part, int64_t part_cap, double *out, hipStream_t s) {
  const int64_t ab = (int64_t)a * b;
  if (ab == 0) return hipSuccess;
  const int tiles = ((a + GR_T - 1) / GR_T) * ((b + GR_T - 1) / GR_T);
  int64_t nchunks = (N + 4095) / 4096;
  // enough blocks to fill the chip, bounded by the partial buffer
  if (nchunks * tiles < 2048) nchunks = (2048 + tiles - 1) / tiles;
  int64_t maxc = (N + GR_ROWS - 1) / GR_ROWS;
  if (nchunks > maxc) nchunks = maxc;
  if (nchunks < 1) nchunks = 1;
  if (nchunks * ab > part_cap) nchunks = part_cap / ab;
  if (nchunks < 1) return hipErrorInvalidValue;
  int64_t rpc = (N + nchunks - 1) / nchunks;
  rpc = ((rpc + GR_ROWS - 1) / GR_ROWS) * GR_ROWS;
  if (rpc < GR_ROWS) rpc = GR_ROWS;
  nchunks = N > 0 ? (N + rpc - 1) / rpc : 1;
  if (N == 0) {
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((ab + 255) / 256)), dim3(256), 0, s,
                       (int64_t)0, ab, part, out);
    return hipGetLastError();
  }
  dim3 grid((a + GR_T - 1) / GR_T, (b + GR_T - 1) / GR_T, (unsigned)nchunks);
  hipLaunchKernelGGL((k_gram<T>), grid, dim3(256), 0, s, N, a, X, ldx, b, Y, ldy, rpc, part);
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((ab + 255) / 256)), dim3(256), 0, s, nchunks,
                     ab, part, out);
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

template <typename T>
hipError_t launch_gemm_ts(int64_t N, int a, const T *X, int ldx, int b, const double *M, int ldm,
                          T *C, int ldc, double beta, hipStream_t s) {
  if (N == 0 || b == 0) return hipSuccess;
  if (a == 0) {  // C = beta C
    if (beta == 1.0) return hipSuccess;
    return launch_axpy<T>(N, b, beta - 1.0, C, ldc, C, ldc, s);
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
  Y[r * ldy + c] = (Tout)X[r * ldx + c];
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
  template hipError_t launch_grad<T>(const Plan &, const T *, const T *, int, const T *, int, int, \
                                     double, T *, int, PassScratch, int64_t *, hipStream_t);       \
  template hipError_t launch_sddmm<T>(const Plan &, const T *, const T *, int, const T *, int,    \
                                      int, T *, PassScratch, hipStream_t);                         \
  template hipError_t launch_spmm<T>(const Plan &, const T *, const T *, int, int, double,         \
                                     const T *, int, int, const T *, int, T *, int, PassScratch,   \
                                     hipStream_t);                                                 \
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
