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
// registers until the row ends.  (Index/value streams use ordinary loads:
// measured on the 1e8-entry workload, non-temporal loads were up to 30%
// slower on the column-oriented passes and no faster elsewhere.)
//
// Determinism: no floating-point atomics anywhere.  Scalar sums are written
// per wave and added in a fixed order by a one-block kernel; long rows are
// split into fixed pieces whose partial rows are added in piece order.
#include <hip/hip_runtime.h>

#include "bmg_internal.h"

namespace bmg {

// Elements per 16-byte lane slice of the gathered type.
template <typename TG> struct VT { static constexpr int V = 16 / (int)sizeof(TG); };

// BF16 storage (upper half of an FP32), rounded to nearest even.
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ bf16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
template <typename To, typename From> __device__ __forceinline__ To cvt(From x) { return (To)x; }
template <> __device__ __forceinline__ float cvt<float, bf16_t>(bf16_t x) { return bf2f(x); }
template <> __device__ __forceinline__ double cvt<double, bf16_t>(bf16_t x) { return (double)bf2f(x); }
template <> __device__ __forceinline__ bf16_t cvt<bf16_t, float>(float x) { return f2bf(x); }
template <> __device__ __forceinline__ bf16_t cvt<bf16_t, double>(double x) { return f2bf((float)x); }

#ifndef BMG_NT_STREAMS
#define BMG_NT_STREAMS 0
#endif
template <typename T>
__device__ __forceinline__ T nt_load(const T *p) {
#if BMG_NT_STREAMS
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

// Load V consecutive elements row[f0 .. f0+V) of memory type TM into T
// registers, with per-element bound lim (elements at or beyond lim read as 0
// and are never touched).
template <typename T, typename TM, int V>
__device__ __forceinline__ void ldv(const TM *__restrict__ row, int f0, int lim, T (&x)[V]) {
  if (f0 + V <= lim) {
    if constexpr (sizeof(TM) == 8 && V == 2) {
      const double2 v = *reinterpret_cast<const double2 *>(row + f0);
      x[0] = (T)v.x; x[1] = (T)v.y;
      return;
    } else if constexpr (sizeof(TM) == 4 && (V == 4 || V == 8)) {
#pragma unroll
      for (int h = 0; h < V / 4; ++h) {
        const float4 v = *reinterpret_cast<const float4 *>(row + f0 + 4 * h);
        x[4 * h] = (T)v.x; x[4 * h + 1] = (T)v.y; x[4 * h + 2] = (T)v.z; x[4 * h + 3] = (T)v.w;
      }
      return;
    } else if constexpr (sizeof(TM) == 2 && V == 8) {
      const uint4 v = *reinterpret_cast<const uint4 *>(row + f0);
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        x[2 * h] = (T)__uint_as_float(w[h] << 16);
        x[2 * h + 1] = (T)__uint_as_float(w[h] & 0xffff0000u);
      }
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < V; ++e) x[e] = (f0 + e < lim) ? cvt<T, TM>(row[f0 + e]) : T(0);
}

template <typename T, typename TM, int V>
__device__ __forceinline__ void stv(TM *__restrict__ row, int f0, int lim, const T (&x)[V]) {
  if (f0 + V <= lim) {
    if constexpr (sizeof(TM) == 8 && sizeof(T) == 8 && V == 2) {
      *reinterpret_cast<double2 *>(row + f0) = make_double2(x[0], x[1]);
      return;
    } else if constexpr (sizeof(TM) == 4 && sizeof(T) == 4 && (V == 4 || V == 8)) {
#pragma unroll
      for (int h = 0; h < V / 4; ++h)
        *reinterpret_cast<float4 *>(row + f0 + 4 * h) =
            make_float4(x[4 * h], x[4 * h + 1], x[4 * h + 2], x[4 * h + 3]);
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < V; ++e)
    if (f0 + e < lim) row[f0 + e] = cvt<TM, T>(x[e]);
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

#ifndef BMG_UNROLL
#define BMG_UNROLL 4
#endif
constexpr int UNROLL = BMG_UNROLL;  // entries in flight per lane group
constexpr int WAVES_PER_BLOCK = 4;

__host__ __device__ inline int64_t short_waves(const Plan &pl, int G) {
  const int S = 64 / G;
  return (pl.n_short + S - 1) / S;
}

// Grid of a row-kernel launch: the short-row waves first, then, from a block
// index that is a multiple of 8, the piece waves.  Blocks are dealt to the 8
// XCDs in turn; piece block bb takes launch slots from run (bb % 8) of the
// piece order, so each XCD works through a contiguous run of column ranges.
__host__ __device__ inline int64_t piece_block0(const Plan &pl, int G) {
  const int64_t sb = (short_waves(pl, G) + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
  return (sb + 7) / 8 * 8;
}
__host__ __device__ inline int64_t piece_blocks(const Plan &pl) {
  return ((pl.n_pieces + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK + 7) / 8 * 8;
}
__host__ __device__ inline int64_t grid_blocks(const Plan &pl, int G) {
  int64_t b = pl.n_pieces == 0
                  ? (short_waves(pl, G) + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK
                  : piece_block0(pl, G) + piece_blocks(pl);
  return b > 0 ? b : 1;
}
// Work of the calling wave: 0 = short-row wave w, 1 = piece w, -1 = none.
__device__ __forceinline__ int wave_work(const Plan &pl, int G, int64_t &w) {
  const int wave = threadIdx.x >> 6;
  const int64_t b = blockIdx.x, pb0 = piece_block0(pl, G);
  if (b < pb0) {
    w = b * WAVES_PER_BLOCK + wave;
    return w < short_waves(pl, G) ? 0 : -1;
  }
  const int64_t nb8 = piece_blocks(pl) / 8, bb = b - pb0;
  const int64_t slot = ((bb % 8) * nb8 + bb / 8) * WAVES_PER_BLOCK + wave;
  if (slot >= pl.n_pieces) return -1;
  w = pl.piece_ord[slot];
  return 1;
}

// ============================================================================ lane-group row access
// A lane group of G lanes owns one row of Omega.  A dense k-vector is split in
// C chunks of G*V consecutive columns (one 128-byte line for G = 8 in FP64);
// lane `sub` holds columns c*G*V + sub*V .. +V-1 of chunk c.
template <typename T, typename TG, int G, int C>
struct Row {
  static constexpr int V = VT<TG>::V;
  static constexpr int CW = G * V;       // columns per chunk
  static constexpr int WB = CW * C;      // columns covered
  T v[C][V];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < V; ++e) v[c][e] = T(0);
  }
  template <typename TM>
  __device__ __forceinline__ void load(const TM *__restrict__ row, int sub, int lim) {
#pragma unroll
    for (int c = 0; c < C; ++c) ldv<T, TM, V>(row, c * CW + sub * V, lim, v[c]);
  }
  template <typename TM>
  __device__ __forceinline__ void store(TM *__restrict__ row, int sub, int lim) const {
#pragma unroll
    for (int c = 0; c < C; ++c) stv<T, TM, V>(row, c * CW + sub * V, lim, v[c]);
  }
  __device__ __forceinline__ T dot(const Row &o) const {
    T s = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < V; ++e) s += v[c][e] * o.v[c][e];
    return s;
  }
  __device__ __forceinline__ void axpy(T a, const Row &o) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < V; ++e) v[c][e] += a * o.v[c][e];
  }
};

// ============================================================================ fused residual + product
// For entries p, p+step, ... (n of them) of one row:
//   r = x . y_j - a_p ;  acc += r y_j ;  ss += r^2   (ss on the group leader only)
template <typename T, typename TG, int G, int C>
__device__ __forceinline__ void grad_block(const Plan &pl, const T *__restrict__ a,
                                           const TG *__restrict__ Y, int ldy, int k, int sub,
                                           const Row<T, TG, G, C> &x, Row<T, TG, G, C> &acc, double &ss,
                                           bool leader, int64_t p, int64_t step, int n) {
  int j[UNROLL];
  T av[UNROLL];
  Row<T, TG, G, C> y[UNROLL];
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
    if (j[u] >= 0) y[u].load(Y + (int64_t)j[u] * ldy, sub, k);
    else y[u].zero();
  }
  T d[UNROLL];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) d[u] = x.dot(y[u]);
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) d[u] = group_sum<G>(d[u]);
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    if (u < n) {
      const T r = d[u] - av[u];
      acc.axpy(r, y[u]);
      if (leader) ss += (double)r * (double)r;
    }
  }
}

template <typename T, typename TG, int G, int C>
__global__ __launch_bounds__(256) void k_grad(Plan pl, const T *__restrict__ a,
                                              const T *__restrict__ X, int ldx,
                                              const TG *__restrict__ Y, int ldy, int k, double lam,
                                              T *__restrict__ Out, int ldo,
                                              T *__restrict__ partial, double *__restrict__ wsum) {
  using RowT = Row<T, TG, G, C>;
  constexpr int S = 64 / G, WB = RowT::WB;
  const int lane = threadIdx.x & 63, slot = lane / G, sub = lane % G;
  const int64_t gw = (int64_t)blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
  int64_t w = 0;
  const int kind = wave_work(pl, G, w);
  const bool leader = (sub == 0);
  double ss = 0.0;
  RowT acc;
  acc.zero();
  if (kind == 0) {
    const int64_t ri = w * S + slot;
    if (ri < pl.n_short) {
      const int row = pl.short_rows[ri];
      RowT x;
      x.load(X + (int64_t)row * ldx, sub, k);
      const int64_t beg = pl.ptr[row], end = pl.ptr[row + 1];
      for (int64_t p = beg; p < end; p += UNROLL) {
        const int n = (int)((end - p) < UNROLL ? (end - p) : UNROLL);
        grad_block<T, TG, G, C>(pl, a, Y, ldy, k, sub, x, acc, ss, leader, p, 1, n);
      }
      acc.axpy((T)lam, x);
      acc.store(Out + (int64_t)row * ldo, sub, k);
    }
  } else if (kind == 1) {
    const int64_t pc = w;
    const int row = pl.piece_row[pc];
    const int64_t beg = pl.piece_beg[pc], end = pl.piece_end[pc];
    RowT x;
    x.load(X + (int64_t)row * ldx, sub, k);
    for (int64_t p = beg + slot; p < end; p += (int64_t)S * UNROLL) {
      const int64_t rem = (end - p + S - 1) / S;
      const int n = (int)(rem < UNROLL ? rem : UNROLL);
      grad_block<T, TG, G, C>(pl, a, Y, ldy, k, sub, x, acc, ss, leader, p, S, n);
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < RowT::V; ++e) acc.v[c][e] = slot_sum<G>(acc.v[c][e]);
    if (slot == 0) acc.store(partial + pc * WB, sub, WB);
  }
  ss = wave_sum(ss);
  if (lane == 0) wsum[gw] = ss;
}

// Long rows: Out_row = sum of piece partials (piece order) + lam * x_row.
template <typename T, typename TG, int G, int C>
__global__ __launch_bounds__(256) void k_grad_fix(Plan pl, const T *__restrict__ partial,
                                                  const T *__restrict__ X, int ldx, int k,
                                                  double lam, T *__restrict__ Out, int ldo) {
  using RowT = Row<T, TG, G, C>;
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  if (g >= pl.n_long) return;
  const int row = pl.long_rows[g];
  RowT acc, t;
  acc.zero();
  for (int pc = pl.long_p0[g]; pc < pl.long_p0[g + 1]; ++pc) {
    t.load(partial + (int64_t)pc * RowT::WB, sub, RowT::WB);
    acc.axpy(T(1), t);
  }
  RowT x;
  x.load(X + (int64_t)row * ldx, sub, k);
  acc.axpy((T)lam, x);
  acc.store(Out + (int64_t)row * ldo, sub, k);
}

// ============================================================================ sampled residual
template <typename T, typename TG, int G, int C>
__device__ __forceinline__ void sddmm_block(const Plan &pl, const T *__restrict__ a,
                                            const TG *__restrict__ Y, int ldy, int k, int sub,
                                            const Row<T, TG, G, C> &x, T *__restrict__ R, double &ss,
                                            double &sx, bool leader, int64_t p, int64_t step,
                                            int n) {
  int j[UNROLL];
  T av[UNROLL];
  Row<T, TG, G, C> y[UNROLL];
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
    if (j[u] >= 0) y[u].load(Y + (int64_t)j[u] * ldy, sub, k);
    else y[u].zero();
  }
  T d[UNROLL];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) d[u] = group_sum<G>(x.dot(y[u]));
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

template <typename T, typename TG, int G, int C>
__global__ __launch_bounds__(256) void k_sddmm(Plan pl, const T *__restrict__ a,
                                               const T *__restrict__ X, int ldx,
                                               const TG *__restrict__ Y, int ldy, int k,
                                               T *__restrict__ R, double *__restrict__ wsum) {
  using RowT = Row<T, TG, G, C>;
  constexpr int S = 64 / G;
  const int lane = threadIdx.x & 63, slot = lane / G, sub = lane % G;
  const int64_t gw = (int64_t)blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
  int64_t w = 0;
  const int kind = wave_work(pl, G, w);
  const bool leader = (sub == 0);
  double ss = 0.0, sx = 0.0;
  if (kind == 0) {
    const int64_t ri = w * S + slot;
    if (ri < pl.n_short) {
      const int row = pl.short_rows[ri];
      RowT x;
      x.load(X + (int64_t)row * ldx, sub, k);
      const int64_t beg = pl.ptr[row], end = pl.ptr[row + 1];
      for (int64_t p = beg; p < end; p += UNROLL) {
        const int n = (int)((end - p) < UNROLL ? (end - p) : UNROLL);
        sddmm_block<T, TG, G, C>(pl, a, Y, ldy, k, sub, x, R, ss, sx, leader, p, 1, n);
      }
    }
  } else if (kind == 1) {
    const int64_t pc = w;
    const int row = pl.piece_row[pc];
    const int64_t beg = pl.piece_beg[pc], end = pl.piece_end[pc];
    RowT x;
    x.load(X + (int64_t)row * ldx, sub, k);
    for (int64_t p = beg + slot; p < end; p += (int64_t)S * UNROLL) {
      const int64_t rem = (end - p + S - 1) / S;
      const int n = (int)(rem < UNROLL ? rem : UNROLL);
      sddmm_block<T, TG, G, C>(pl, a, Y, ldy, k, sub, x, R, ss, sx, leader, p, S, n);
    }
  }
  ss = wave_sum(ss);
  sx = wave_sum(sx);
  if (lane == 0) {
    wsum[2 * gw] = ss;
    wsum[2 * gw + 1] = sx;
  }
}

// ============================================================================ sparse x dense
template <typename T, typename TG, int G, int C>
__device__ __forceinline__ void spmm_block(const Plan &pl, const T *__restrict__ Sv,
                                           const TG *__restrict__ B, int ldb, int wq, int sub,
                                           Row<T, TG, G, C> &acc, int64_t p, int64_t step, int n) {
  int j[UNROLL];
  T sv[UNROLL];
  Row<T, TG, G, C> b[UNROLL];
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
    if (j[u] >= 0) b[u].load(B + (int64_t)j[u] * ldb, sub, wq);
    else b[u].zero();
  }
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) acc.axpy(sv[u], b[u]);
}

// acc <- coef * acc + x_row . M[:, slice]
template <typename T, typename TG, int G, int C>
__device__ __forceinline__ void lowrank_epilogue(Row<T, TG, G, C> &acc, double coef,
                                                 const T *__restrict__ xr, int kx,
                                                 const T *__restrict__ M, int ldm, int wq,
                                                 int sub) {
  using RowT = Row<T, TG, G, C>;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int e = 0; e < RowT::V; ++e) acc.v[c][e] *= (T)coef;
  for (int r = 0; r < kx; ++r) {
    RowT mv;
    mv.load(M + (int64_t)r * ldm, sub, wq);
    acc.axpy(xr[r], mv);
  }
}

template <typename T, typename TG, int G, int C>
__global__ __launch_bounds__(256) void k_spmm(Plan pl, const T *__restrict__ Sv,
                                              const TG *__restrict__ B, int ldb, int wq,
                                              double coef, const T *__restrict__ X, int ldx,
                                              int kx, const T *__restrict__ M, int ldm,
                                              T *__restrict__ Cm, int ldc,
                                              T *__restrict__ partial) {
  using RowT = Row<T, TG, G, C>;
  constexpr int S = 64 / G, WB = RowT::WB;
  const int lane = threadIdx.x & 63, slot = lane / G, sub = lane % G;
  int64_t w = 0;
  const int kind = wave_work(pl, G, w);
  RowT acc;
  acc.zero();
  if (kind == 0) {
    const int64_t ri = w * S + slot;
    if (ri < pl.n_short) {
      const int row = pl.short_rows[ri];
      const int64_t beg = pl.ptr[row], end = pl.ptr[row + 1];
      for (int64_t p = beg; p < end; p += UNROLL) {
        const int n = (int)((end - p) < UNROLL ? (end - p) : UNROLL);
        spmm_block<T, TG, G, C>(pl, Sv, B, ldb, wq, sub, acc, p, 1, n);
      }
      lowrank_epilogue<T, TG, G, C>(acc, coef, X + (int64_t)row * ldx, kx, M, ldm, wq, sub);
      acc.store(Cm + (int64_t)row * ldc, sub, wq);
    }
  } else if (kind == 1) {
    const int64_t pc = w;
    const int64_t beg = pl.piece_beg[pc], end = pl.piece_end[pc];
    for (int64_t p = beg + slot; p < end; p += (int64_t)S * UNROLL) {
      const int64_t rem = (end - p + S - 1) / S;
      const int n = (int)(rem < UNROLL ? rem : UNROLL);
      spmm_block<T, TG, G, C>(pl, Sv, B, ldb, wq, sub, acc, p, S, n);
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < RowT::V; ++e) acc.v[c][e] = slot_sum<G>(acc.v[c][e]);
    if (slot == 0) acc.store(partial + pc * WB, sub, WB);
  }
}

template <typename T, typename TG, int G, int C>
__global__ __launch_bounds__(256) void k_spmm_fix(Plan pl, const T *__restrict__ partial,
                                                  double coef, const T *__restrict__ X, int ldx,
                                                  int kx, const T *__restrict__ M, int ldm, int wq,
                                                  T *__restrict__ Cm, int ldc) {
  using RowT = Row<T, TG, G, C>;
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int sub = threadIdx.x % G;
  if (g >= pl.n_long) return;
  const int row = pl.long_rows[g];
  RowT acc, t;
  acc.zero();
  for (int pc = pl.long_p0[g]; pc < pl.long_p0[g + 1]; ++pc) {
    t.load(partial + (int64_t)pc * RowT::WB, sub, RowT::WB);
    acc.axpy(T(1), t);
  }
  lowrank_epilogue<T, TG, G, C>(acc, coef, X + (int64_t)row * ldx, kx, M, ldm, wq, sub);
  acc.store(Cm + (int64_t)row * ldc, sub, wq);
}

// ============================================================================ launchers
// Lane group G and chunk count C for a width w (V elements of the gathered type
// per lane): G = 2 or 4 for narrow rows (one partial line), else G = 8 with
// C = ceil(w / (8 V)) line-sized chunks.
struct GC {
  int G, C;
};
static inline GC pick_gc(int width, int V) {
  if (width <= 2 * V) return {2, 1};
  if (width <= 4 * V) return {4, 1};
  int c = (width + 8 * V - 1) / (8 * V);
  return {8, c < 1 ? 1 : c};
}


#define BMG_DISPATCH_GC(gc, ...)                                                        \
  do {                                                                                  \
    if (gc.G == 2) { constexpr int GG = 2, CC = 1; __VA_ARGS__; }                       \
    else if (gc.G == 4) { constexpr int GG = 4, CC = 1; __VA_ARGS__; }                  \
    else switch (gc.C) {                                                                \
      case 1: { constexpr int GG = 8, CC = 1; __VA_ARGS__; } break;                     \
      case 2: { constexpr int GG = 8, CC = 2; __VA_ARGS__; } break;                     \
      case 3: { constexpr int GG = 8, CC = 3; __VA_ARGS__; } break;                     \
      case 4: { constexpr int GG = 8, CC = 4; __VA_ARGS__; } break;                     \
      case 5: { constexpr int GG = 8, CC = 5; __VA_ARGS__; } break;                     \
      case 6: { constexpr int GG = 8, CC = 6; __VA_ARGS__; } break;                     \
      case 7: { constexpr int GG = 8, CC = 7; __VA_ARGS__; } break;                     \
      default: { constexpr int GG = 8, CC = 8; __VA_ARGS__; } break;                    \
    }                                                                                   \
  } while (0)

// Each launch writes one scalar slot (or pair) per wave of its grid, idle
// waves included, and reduces them in wave order.
template <typename T, typename TG>
hipError_t launch_grad(const Plan &pl, const T *a, const T *X, int ldx, const TG *Y, int ldy, int k,
                       double lam, T *Out, int ldo, PassScratch sc, int64_t *waves_out,
                       hipStream_t s) {
  constexpr int V = VT<TG>::V;
  if (k > max_width<T>()) return hipErrorInvalidValue;
  const GC gc = pick_gc(k, V);
  const int64_t nb = grid_blocks(pl, gc.G), waves = nb * WAVES_PER_BLOCK;
  if (sc.ev0) (void)hipEventRecord(sc.ev0, s);
  BMG_DISPATCH_GC(gc, {
    hipLaunchKernelGGL((k_grad<T, TG, GG, CC>), dim3((unsigned)nb), dim3(256), 0, s, pl, a, X, ldx,
                       Y, ldy, k, lam, Out, ldo, (T *)sc.partial, sc.wsum);
    if (pl.n_long > 0) {
      const int64_t thr = pl.n_long * GG;
      hipLaunchKernelGGL((k_grad_fix<T, TG, GG, CC>), dim3((unsigned)((thr + 255) / 256)),
                         dim3(256), 0, s, pl, (const T *)sc.partial, X, ldx, k, lam, Out, ldo);
    }
  });
  if (sc.ev1) (void)hipEventRecord(sc.ev1, s);
  if (waves_out) *waves_out = waves;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_wsum(sc.wsum, waves, 1, sc.wpart, sc.result, s);
}

template <typename T, typename TG>
hipError_t launch_sddmm(const Plan &pl, const T *a, const T *X, int ldx, const TG *Y, int ldy, int k,
                        T *R, PassScratch sc, hipStream_t s) {
  constexpr int V = VT<TG>::V;
  if (k > max_width<T>()) return hipErrorInvalidValue;
  const GC gc = pick_gc(k, V);
  const int64_t nb = grid_blocks(pl, gc.G), waves = nb * WAVES_PER_BLOCK;
  if (sc.ev0) (void)hipEventRecord(sc.ev0, s);
  BMG_DISPATCH_GC(gc, {
    hipLaunchKernelGGL((k_sddmm<T, TG, GG, CC>), dim3((unsigned)nb), dim3(256), 0, s, pl, a, X,
                       ldx, Y, ldy, k, R, sc.wsum);
  });
  if (sc.ev1) (void)hipEventRecord(sc.ev1, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_wsum(sc.wsum, waves, 2, sc.wpart, sc.result, s);
}

template <typename T, typename TG>
hipError_t launch_spmm(const Plan &pl, const T *Sv, const TG *B, int ldb, int q, double coef,
                       const T *X, int ldx, int kx, const T *M, int ldm, T *Cm, int ldc,
                       PassScratch sc, hipStream_t s) {
  constexpr int V = VT<TG>::V;
  const int WMAX = max_width<T>();
  if (sc.ev0) (void)hipEventRecord(sc.ev0, s);
  for (int c0 = 0; c0 < q; c0 += WMAX) {
    const int wq = (q - c0) < WMAX ? (q - c0) : WMAX;
    const GC gc = pick_gc(wq, V);
    const int64_t nb = grid_blocks(pl, gc.G);
    BMG_DISPATCH_GC(gc, {
      hipLaunchKernelGGL((k_spmm<T, TG, GG, CC>), dim3((unsigned)nb), dim3(256), 0, s, pl, Sv,
                         B + c0, ldb, wq, coef, X, ldx, kx, M ? M + c0 : M, ldm, Cm + c0, ldc,
                         (T *)sc.partial);
      if (pl.n_long > 0) {
        const int64_t thr = pl.n_long * GG;
        hipLaunchKernelGGL((k_spmm_fix<T, TG, GG, CC>), dim3((unsigned)((thr + 255) / 256)),
                           dim3(256), 0, s, pl, (const T *)sc.partial, coef, X, ldx, kx,
                           M ? M + c0 : M, ldm, wq, Cm + c0, ldc);
      }
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (sc.ev1) (void)hipEventRecord(sc.ev1, s);
  return hipSuccess;
}

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
  const int ny = ((TA + 3) / 4) * ((TB + 3) / 4);
  int64_t nx = (N + 255) / 256;                 // >= 256 rows per block
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
#define BMG_INST_PASS(T, TG)                                                                    \
  template hipError_t launch_grad<T, TG>(const Plan &, const T *, const T *, int, const TG *, int,   \
                                         int, double, T *, int, PassScratch, int64_t *,              \
                                         hipStream_t);                                               \
  template hipError_t launch_sddmm<T, TG>(const Plan &, const T *, const T *, int, const TG *, int,  \
                                          int, T *, PassScratch, hipStream_t);                       \
  template hipError_t launch_spmm<T, TG>(const Plan &, const T *, const TG *, int, int, double,      \
                                         const T *, int, int, const T *, int, T *, int, PassScratch, \
                                         hipStream_t);
BMG_INST_PASS(double, double)
BMG_INST_PASS(float, float)
BMG_INST_PASS(float, bf16_t)
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
