// Row kernels of the sparse passes (gfx950, wave64) of the BM-Global
// matrix-completion hot path, and their launchers.  Included by one source
// per element type pair (pass_f64.hip, pass_f32.hip, pass_bf16.hip).
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
// per wave and added in a fixed order by a two-stage reduction; long rows are
// split into fixed pieces whose partial rows are added in piece order.
#pragma once
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
    } else if constexpr (sizeof(TM) == 4 && V == 2) {
      const float2 v = *reinterpret_cast<const float2 *>(row + f0);
      x[0] = (T)v.x; x[1] = (T)v.y;
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
    } else if constexpr (sizeof(TM) == 4 && sizeof(T) == 4 && V == 2) {
      *reinterpret_cast<float2 *>(row + f0) = make_float2(x[0], x[1]);
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
// Waves per SIMD the compiler is asked to fit for a row kernel (1: its own
// choice).  The FP64 width-32 passes of the BM phase sit just above a wave
// boundary (98 and 83 VGPRs); asked for one wave more, they fit without spills.
template <typename T, int G, int C> constexpr int grad_waves() { return (sizeof(T) == 8 && G == 8 && C == 2) ? 5 : 1; }
template <typename T, int G, int C> constexpr int sddmm_waves() { return (sizeof(T) == 8 && G == 8 && C == 2) ? 6 : 1; }

// Short rows: a team of max(8, G) lanes per row, 64 / team rows per wave.
__host__ __device__ inline int64_t short_waves(const Plan &pl, int G) {
  const int S = 64 / (G > 8 ? G : 8);
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
// Work of the calling wave of block b: 0 = short-row wave w, 1 = piece w, -1 = none.
__device__ __forceinline__ int wave_work(const Plan &pl, int G, int64_t b, int64_t &w) {
  const int wave = threadIdx.x >> 6;
  const int64_t pb0 = piece_block0(pl, G);
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
// lane `sub` holds columns c*G*V + sub*V .. +V-1 of chunk c.  In a thin row
// (TT) the last chunk is half as wide: lane `sub` holds V/2 columns of it, from
// (C-1)*G*V + sub*V/2; a width just past a whole number of chunks then keeps
// V/2 fewer registers per lane for every row in flight.
template <typename T, typename TG, int G, int C, bool TT = false>
struct Row {
  static constexpr int V = VT<TG>::V;
  static constexpr int CW = G * V;       // columns per chunk
  static constexpr int WB = CW * C;      // columns covered
  // elements per lane of chunk c
  static constexpr __host__ __device__ int vw(int c) { return (TT && c == C - 1) ? V / 2 : V; }
  T v[C][V];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < vw(c); ++e) v[c][e] = T(0);
  }
  template <typename TM>
  __device__ __forceinline__ void load(const TM *__restrict__ row, int sub, int lim) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (TT && c == C - 1) {
        T h[V / 2];
        ldv<T, TM, V / 2>(row, c * CW + sub * (V / 2), lim, h);
#pragma unroll
        for (int e = 0; e < V / 2; ++e) v[c][e] = h[e];
      } else {
        ldv<T, TM, V>(row, c * CW + sub * V, lim, v[c]);
      }
    }
  }
  template <typename TM>
  __device__ __forceinline__ void store(TM *__restrict__ row, int sub, int lim) const {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (TT && c == C - 1) {
        T h[V / 2];
#pragma unroll
        for (int e = 0; e < V / 2; ++e) h[e] = v[c][e];
        stv<T, TM, V / 2>(row, c * CW + sub * (V / 2), lim, h);
      } else {
        stv<T, TM, V>(row, c * CW + sub * V, lim, v[c]);
      }
    }
  }
  __device__ __forceinline__ T dot(const Row &o) const {
    T s = T(0);
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < vw(c); ++e) s += v[c][e] * o.v[c][e];
    return s;
  }
  __device__ __forceinline__ void axpy(T a, const Row &o) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < vw(c); ++e) v[c][e] += a * o.v[c][e];
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
    // entries past the block read entry p (always valid) and are masked out
    const int64_t pp = p + (u < n ? u * step : 0);
    const int jv = nt_load(pl.idx + pp);
    const T avv = nt_load(a + pp);
    j[u] = u < n ? jv : -1;
    av[u] = u < n ? avv : T(0);
  }
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) y[u].load(Y + (int64_t)(j[u] < 0 ? 0 : j[u]) * ldy, sub, k);
  T d[UNROLL];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) d[u] = x.dot(y[u]);
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) d[u] = group_sum<G>(d[u]);
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    const T r = d[u] - av[u];
    acc.axpy(u < n ? r : T(0), y[u]);
    if (leader && u < n) ss += (double)r * (double)r;
  }
}

// ============================================================================ short rows
// A team of TL = max(8, G) lanes owns one short row.  The team loads the row's
// indices and values TL at a time (one cache line per load instruction) and
// hands each entry to one of its E = TL / G lane groups by a lane shuffle; each
// group gathers and accumulates its entries (UNROLL in flight), and the groups'
// rows are added at the end of the row.  Entry e of a chunk goes to group
// e % E; lane e % TL of the team loaded it in load slot e / TL.
template <int G> struct Team {
  static constexpr int TL = G > 8 ? G : 8;              // lanes per row
  static constexpr int E = TL / G;                      // groups per row
  static constexpr int LPL = (UNROLL + G - 1) / G;      // loads per lane per chunk
  static constexpr int CH = TL * LPL;                   // entries per chunk
  static constexpr int NI = CH / E;                     // entries per group per chunk
};

enum TeamMode { TM_GRAD = 0, TM_SDDMM = 1, TM_SPMM = 2 };

// GRAD: acc += r y, ss += r^2 with r = x.y - a;  SDDMM: R = r, ss += r^2,
// sx += r (x.y);  SPMM: acc += a y.  On return every group of the team holds
// the row's sum in acc; ss / sx are held by the group leaders.
template <typename T, typename TG, int G, int C, int MODE, bool TT = false>
__device__ __forceinline__ void team_row(const Plan &pl, int row, const T *__restrict__ a,
                                         const TG *__restrict__ Y, int ldy, int width,
                                         const Row<T, TG, G, C, TT> &x, Row<T, TG, G, C, TT> &acc,
                                         T *__restrict__ R, double &ss, double &sx, int tbase,
                                         int tl) {
  using TM = Team<G>;
  using RowT = Row<T, TG, G, C, TT>;
  const int eg = tl / G, sub = tl % G;
  const bool leader = (sub == 0);
  const int64_t beg = pl.ptr[row], end = pl.ptr[row + 1];
  for (int64_t p0 = beg; p0 < end; p0 += TM::CH) {
    int jl[TM::LPL];
    T al[TM::LPL];
#pragma unroll
    for (int l = 0; l < TM::LPL; ++l) {
      // entries past the row read its last entry (valid) and are masked out
      const int64_t pe = p0 + l * TM::TL + tl;
      const int64_t pc = pe < end ? pe : end - 1;
      const int jv = nt_load(pl.idx + pc);
      const T avv = a ? nt_load(a + pc) : T(0);
      jl[l] = pe < end ? jv : -1;
      al[l] = pe < end ? avv : T(0);
    }
    // batches stay rolled (UNROLL gathers in flight are enough); only G = 2
    // has two load slots, and it has a single batch
    static_assert(TM::LPL == 1 || TM::NI <= UNROLL, "load slot must be known at compile time");
#pragma unroll 1
    for (int i0 = 0; i0 < TM::NI; i0 += UNROLL) {
      int j[UNROLL];
      T av[UNROLL];
      RowT y[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int eo = TM::E * (i0 + u);       // chunk offset of this step's group-0 entry
        if (i0 + u < TM::NI) {
          const int src = tbase + eg + eo % TM::TL;
          j[u] = __shfl(jl[TM::LPL == 1 ? 0 : eo / TM::TL], src, 64);
          av[u] = __shfl(al[TM::LPL == 1 ? 0 : eo / TM::TL], src, 64);
        } else {
          j[u] = -1;
          av[u] = T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u)
        y[u].load(Y + (int64_t)(j[u] < 0 ? 0 : j[u]) * ldy, sub, width);
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        if (MODE == TM_SPMM) {
          acc.axpy(av[u], y[u]);
        } else {
          const T d = group_sum<G>(x.dot(y[u]));
          const T res = d - av[u];
          if (MODE == TM_GRAD) acc.axpy(j[u] >= 0 ? res : T(0), y[u]);
          if (leader && j[u] >= 0) {
            if (MODE == TM_SDDMM && R) R[p0 + eg + TM::E * (i0 + u)] = res;
            ss += (double)res * (double)res;
            if (MODE == TM_SDDMM) sx += (double)res * (double)d;
          }
        }
      }
    }
  }
  if (MODE != TM_SDDMM && TM::E > 1) {
#pragma unroll
    for (int o = G; o < TM::TL; o <<= 1)
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < RowT::vw(c); ++e) acc.v[c][e] += __shfl_xor(acc.v[c][e], o, 64);
  }
}

// Fused residual + product pass; blk is the block's index within its pass.
template <typename T, typename TG, int G, int C>
__device__ __forceinline__ void grad_body(const Plan &pl, int64_t blk, const T *__restrict__ a,
                                          const T *__restrict__ X, int ldx,
                                          const TG *__restrict__ Y, int ldy, int k, double lam,
                                          T *__restrict__ Out, int ldo, T *__restrict__ partial,
                                          double *__restrict__ wsum) {
  using RowT = Row<T, TG, G, C>;
  constexpr int S = 64 / G, WB = RowT::WB;
  const int lane = threadIdx.x & 63, slot = lane / G, sub = lane % G;
  const int64_t gw = blk * WAVES_PER_BLOCK + (threadIdx.x >> 6);
  int64_t w = 0;
  const int kind = wave_work(pl, G, blk, w);
  const bool leader = (sub == 0);
  double ss = 0.0;
  RowT acc;
  acc.zero();
  if (kind == 0) {
    constexpr int TL = Team<G>::TL;
    const int team = lane / TL, tl = lane % TL;
    const int64_t ri = w * (64 / TL) + team;
    if (ri < pl.n_short) {
      const int row = pl.short_rows[ri];
      RowT x;
      x.load(X + (int64_t)row * ldx, sub, k);
      double sx = 0.0;
      team_row<T, TG, G, C, TM_GRAD>(pl, row, a, Y, ldy, k, x, acc, (T *)nullptr, ss, sx,
                                     team * TL, tl);
      if (tl < G) {
        acc.axpy((T)lam, x);
        acc.store(Out + (int64_t)row * ldo, sub, k);
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
template <typename T, typename TG, int G, int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(grad_waves<T, G, C>()))) void k_grad(Plan pl, const T *__restrict__ a,
                                              const T *__restrict__ X, int ldx,
                                              const TG *__restrict__ Y, int ldy, int k, double lam,
                                              T *__restrict__ Out, int ldo,
                                              T *__restrict__ partial, double *__restrict__ wsum) {
  grad_body<T, TG, G, C>(pl, blockIdx.x, a, X, ldx, Y, ldy, k, lam, Out, ldo, partial, wsum);
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
    const int64_t pp = p + (u < n ? u * step : 0);
    const int jv = nt_load(pl.idx + pp);
    const T avv = a ? nt_load(a + pp) : T(0);
    j[u] = u < n ? jv : -1;
    av[u] = u < n ? avv : T(0);
  }
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) y[u].load(Y + (int64_t)(j[u] < 0 ? 0 : j[u]) * ldy, sub, k);
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
__device__ __forceinline__ void sddmm_body(const Plan &pl, int64_t blk, const T *__restrict__ a,
                                           const T *__restrict__ X, int ldx,
                                           const TG *__restrict__ Y, int ldy, int k,
                                           T *__restrict__ R, double *__restrict__ wsum) {
  using RowT = Row<T, TG, G, C>;
  constexpr int S = 64 / G;
  const int lane = threadIdx.x & 63, slot = lane / G, sub = lane % G;
  const int64_t gw = blk * WAVES_PER_BLOCK + (threadIdx.x >> 6);
  int64_t w = 0;
  const int kind = wave_work(pl, G, blk, w);
  const bool leader = (sub == 0);
  double ss = 0.0, sx = 0.0;
  if (kind == 0) {
    constexpr int TL = Team<G>::TL;
    const int team = lane / TL, tl = lane % TL;
    const int64_t ri = w * (64 / TL) + team;
    if (ri < pl.n_short) {
      // a plan without a row list takes the rows in their own order
      const int row = pl.short_rows ? pl.short_rows[ri] : (int)ri;
      RowT x, acc;
      x.load(X + (int64_t)row * ldx, sub, k);
      team_row<T, TG, G, C, TM_SDDMM>(pl, row, a, Y, ldy, k, x, acc, R, ss, sx, team * TL, tl);
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
template <typename T, typename TG, int G, int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sddmm_waves<T, G, C>()))) void k_sddmm(Plan pl, const T *__restrict__ a,
                                               const T *__restrict__ X, int ldx,
                                               const TG *__restrict__ Y, int ldy, int k,
                                               T *__restrict__ R, double *__restrict__ wsum) {
  sddmm_body<T, TG, G, C>(pl, blockIdx.x, a, X, ldx, Y, ldy, k, R, wsum);
}

// ============================================================================ sparse x dense
template <typename T, typename TG, int G, int C, bool TT = false>
__device__ __forceinline__ void spmm_block(const Plan &pl, const T *__restrict__ Sv,
                                           const TG *__restrict__ B, int ldb, int wq, int sub,
                                           Row<T, TG, G, C, TT> &acc, int64_t p, int64_t step, int n) {
  int j[UNROLL];
  T sv[UNROLL];
  Row<T, TG, G, C, TT> b[UNROLL];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) {
    const int64_t pp = p + (u < n ? u * step : 0);
    const int jv = nt_load(pl.idx + pp);
    const T svv = nt_load(Sv + pp);
    j[u] = u < n ? jv : -1;
    sv[u] = u < n ? svv : T(0);
  }
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) b[u].load(B + (int64_t)(j[u] < 0 ? 0 : j[u]) * ldb, sub, wq);
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) acc.axpy(sv[u], b[u]);
}

// acc <- coef * acc + x_row . M[:, slice]
template <typename T, typename TG, int G, int C, bool TT = false>
__device__ __forceinline__ void lowrank_epilogue(Row<T, TG, G, C, TT> &acc, double coef,
                                                 const T *__restrict__ xr, int kx,
                                                 const T *__restrict__ M, int ldm, int wq,
                                                 int sub) {
  using RowT = Row<T, TG, G, C, TT>;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int e = 0; e < RowT::vw(c); ++e) acc.v[c][e] *= (T)coef;
  for (int r = 0; r < kx; ++r) {
    RowT mv;
    mv.load(M + (int64_t)r * ldm, sub, wq);
    acc.axpy(xr[r], mv);
  }
}

template <typename T, typename TG, int G, int C, bool TT = false>
__device__ __forceinline__ void spmm_body(const Plan &pl, int64_t blk, const T *__restrict__ Sv,
                                              const TG *__restrict__ B, int ldb, int wq,
                                              double coef, const T *__restrict__ X, int ldx,
                                              int kx, const T *__restrict__ M, int ldm,
                                              T *__restrict__ Cm, int ldc,
                                              T *__restrict__ partial) {
  using RowT = Row<T, TG, G, C, TT>;
  constexpr int S = 64 / G, WB = RowT::WB;
  const int lane = threadIdx.x & 63, slot = lane / G, sub = lane % G;
  int64_t w = 0;
  const int kind = wave_work(pl, G, blk, w);
  RowT acc;
  acc.zero();
  if (kind == 0) {
    constexpr int TL = Team<G>::TL;
    const int team = lane / TL, tl = lane % TL;
    const int64_t ri = w * (64 / TL) + team;
    if (ri < pl.n_short) {
      const int row = pl.short_rows[ri];
      RowT none;
      double s0 = 0.0, s1 = 0.0;
      team_row<T, TG, G, C, TM_SPMM, TT>(pl, row, Sv, B, ldb, wq, none, acc, (T *)nullptr, s0, s1,
                                     team * TL, tl);
      if (tl < G) {
        lowrank_epilogue<T, TG, G, C, TT>(acc, coef, X + (int64_t)row * ldx, kx, M, ldm, wq, sub);
        acc.store(Cm + (int64_t)row * ldc, sub, wq);
      }
    }
  } else if (kind == 1) {
    const int64_t pc = w;
    const int64_t beg = pl.piece_beg[pc], end = pl.piece_end[pc];
    for (int64_t p = beg + slot; p < end; p += (int64_t)S * UNROLL) {
      const int64_t rem = (end - p + S - 1) / S;
      const int n = (int)(rem < UNROLL ? rem : UNROLL);
      spmm_block<T, TG, G, C, TT>(pl, Sv, B, ldb, wq, sub, acc, p, S, n);
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int e = 0; e < RowT::vw(c); ++e) acc.v[c][e] = slot_sum<G>(acc.v[c][e]);
    if (slot == 0) acc.store(partial + pc * WB, sub, WB);
  }
}

template <typename T, typename TG, int G, int C, bool TT>
__global__ __launch_bounds__(256) void k_spmm(Plan pl, const T *__restrict__ Sv,
                                              const TG *__restrict__ B, int ldb, int wq,
                                              double coef, const T *__restrict__ X, int ldx,
                                              int kx, const T *__restrict__ M, int ldm,
                                              T *__restrict__ Cm, int ldc,
                                              T *__restrict__ partial) {
  spmm_body<T, TG, G, C, TT>(pl, blockIdx.x, Sv, B, ldb, wq, coef, X, ldx, kx, M, ldm, Cm, ldc, partial);
}

// Thin rows keep few enough registers for six waves per SIMD; the hint lets the
// compiler fit the last few.
template <typename T, typename TG, int G, int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_spmm_thin(
    Plan pl, const T *__restrict__ Sv, const TG *__restrict__ B, int ldb, int wq, double coef,
    const T *__restrict__ X, int ldx, int kx, const T *__restrict__ M, int ldm, T *__restrict__ Cm, int ldc,
    T *__restrict__ partial) {
  spmm_body<T, TG, G, C, true>(pl, blockIdx.x, Sv, B, ldb, wq, coef, X, ldx, kx, M, ldm, Cm, ldc, partial);
}

template <typename T, typename TG, int G, int C, bool TT>
__global__ __launch_bounds__(256) void k_spmm_fix(Plan pl, const T *__restrict__ partial,
                                                  double coef, const T *__restrict__ X, int ldx,
                                                  int kx, const T *__restrict__ M, int ldm, int wq,
                                                  T *__restrict__ Cm, int ldc) {
  using RowT = Row<T, TG, G, C, TT>;
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
  lowrank_epilogue<T, TG, G, C, TT>(acc, coef, X + (int64_t)row * ldx, kx, M, ldm, wq, sub);
  acc.store(Cm + (int64_t)row * ldc, sub, wq);
}

// ============================================================================ launchers
// Lane group G and chunk count C for a width w (V elements of the gathered type
// per lane): G = 2 or 4 for narrow rows (one partial line), G = 8 with
// C = ceil(w / (8 V)) line-sized chunks up to 4 chunks, beyond that G = 16 with
// C = ceil(w / (16 V)) two-line chunks.
struct GC {
  int G, C;
};
static inline GC pick_gc(int width, int V) {
  if (width <= 2 * V) return {2, 1};
  if (width <= 4 * V) return {4, 1};
  if (width <= 32 * V) {
    const int c = (width + 8 * V - 1) / (8 * V);
    return {8, c < 1 ? 1 : c};
  }
  // wider rows: 16-lane groups keep the per-lane registers (and so the
  // occupancy) of at most 4 chunks up to 64 V columns
  const int c = (width + 16 * V - 1) / (16 * V);
  return {16, c < 3 ? 3 : c};
}
// bytes of one piece's partial row for a launch of geometry gc
template <typename T, typename TG>
static inline int64_t partial_row_bytes(const GC &gc) {
  return (int64_t)gc.G * VT<TG>::V * gc.C * (int64_t)sizeof(T);
}


#define BMG_DISPATCH_GC(gc, ...)                                                        \
  do {                                                                                  \
    if (gc.G == 2) { constexpr int GG = 2, CC = 1; __VA_ARGS__; }                       \
    else if (gc.G == 4) { constexpr int GG = 4, CC = 1; __VA_ARGS__; }                  \
    else if (gc.G == 16) switch (gc.C) {                                                \
      case 3: { constexpr int GG = 16, CC = 3; __VA_ARGS__; } break;                    \
      case 4: { constexpr int GG = 16, CC = 4; __VA_ARGS__; } break;                    \
      case 5: { constexpr int GG = 16, CC = 5; __VA_ARGS__; } break;                    \
      case 6: { constexpr int GG = 16, CC = 6; __VA_ARGS__; } break;                    \
      case 7: { constexpr int GG = 16, CC = 7; __VA_ARGS__; } break;                    \
      default: { constexpr int GG = 16, CC = 8; __VA_ARGS__; } break;                   \
    }                                                                                   \
    else switch (gc.C) {                                                                \
      case 1: { constexpr int GG = 8, CC = 1; __VA_ARGS__; } break;                     \
      case 2: { constexpr int GG = 8, CC = 2; __VA_ARGS__; } break;                     \
      case 3: { constexpr int GG = 8, CC = 3; __VA_ARGS__; } break;                     \
      default: { constexpr int GG = 8, CC = 4; __VA_ARGS__; } break;                    \
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
  if (pl.n_pieces * partial_row_bytes<T, TG>(gc) > sc.partial_bytes) return hipErrorInvalidValue;
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
    if (pl.n_pieces * partial_row_bytes<T, TG>(gc) > sc.partial_bytes) return hipErrorInvalidValue;
    const int64_t nb = grid_blocks(pl, gc.G);
    // FP64 and FP32 widths at most half a chunk past a whole number of chunks
    // (q = 2k + 1 of the subspace iteration, say) use thin rows: fewer registers
    // per row in flight, so more waves per SIMD (two or three chunks: wider thin
    // rows would still spill at six waves)
    constexpr bool same = sizeof(T) == sizeof(TG);
    const bool thin = same && gc.C >= 2 && gc.C <= 3 && wq - (gc.C - 1) * gc.G * V <= gc.G * V / 2;
#define BMG_SPMM_LAUNCH(TTv)                                                                          \
  do {                                                                                                \
    if (TTv)                                                                                          \
      hipLaunchKernelGGL((k_spmm_thin<T, TG, GG, CC>), dim3((unsigned)nb), dim3(256), 0, s, pl, Sv,   \
                         B + c0, ldb, wq, coef, X, ldx, kx, M ? M + c0 : M, ldm, Cm + c0, ldc,       \
                         (T *)sc.partial);                                                           \
    else                                                                                              \
      hipLaunchKernelGGL((k_spmm<T, TG, GG, CC, false>), dim3((unsigned)nb), dim3(256), 0, s, pl, Sv, \
                         B + c0, ldb, wq, coef, X, ldx, kx, M ? M + c0 : M, ldm, Cm + c0, ldc,       \
                         (T *)sc.partial);                                                           \
    if (pl.n_long > 0) {                                                                              \
      const int64_t thr = pl.n_long * GG;                                                             \
      hipLaunchKernelGGL((k_spmm_fix<T, TG, GG, CC, TTv>), dim3((unsigned)((thr + 255) / 256)),      \
                         dim3(256), 0, s, pl, (const T *)sc.partial, coef, X, ldx, kx,               \
                         M ? M + c0 : M, ldm, wq, Cm + c0, ldc);                                     \
    }                                                                                                 \
  } while (0)
    BMG_DISPATCH_GC(gc, {
      if constexpr (CC >= 2 && CC <= 3 && same) {
        if (thin) BMG_SPMM_LAUNCH(true);
        else BMG_SPMM_LAUNCH(false);
      } else {
        BMG_SPMM_LAUNCH(false);
      }
    });
#undef BMG_SPMM_LAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (sc.ev1) (void)hipEventRecord(sc.ev1, s);
  return hipSuccess;
}

// ============================================================================ batched passes
// Blocks [b0[d], b0[d+1]) of the grid run pass d; each pass keeps its own block
// numbering (so its wave-to-work mapping, and its results, do not depend on
// the other passes of the launch).
template <typename T, typename TG, int G, int C, int MODE>
__global__ __launch_bounds__(256) void k_batch(BatchArg<T, TG> A) {
  int d = 0;
  while (d + 1 < A.nd && (int64_t)blockIdx.x >= A.b0[d + 1]) ++d;
  const PassArg<T, TG> &D = A.d[d];
  const int64_t blk = (int64_t)blockIdx.x - A.b0[d];
  if (blk >= grid_blocks(D.pl, G)) return;   // padding to a multiple of 8 blocks
  if (MODE == 0)
    grad_body<T, TG, G, C>(D.pl, blk, D.a, D.X, D.ldx, D.Y, D.ldy, D.width, D.lam, D.out, D.ldo,
                           D.partial, D.wsum);
  else if (MODE == 1)
    sddmm_body<T, TG, G, C>(D.pl, blk, D.a, D.X, D.ldx, D.Y, D.ldy, D.width, D.out, D.wsum);
  else
    spmm_body<T, TG, G, C>(D.pl, blk, D.a, D.Y, D.ldy, D.width, D.coef, D.X, D.ldx, D.kx, D.M,
                           D.ldm, D.out, D.ldo, D.partial);
}

// Block d sums the nsum interleaved per-wave slots of pass d in the order of
// launch_reduce_wsum (runs of at least 1024 waves, at most 256 runs, each run
// thread-strided then a binary tree, then the same over the run sums), so a
// batched pass reports bit for bit what it reports alone.
template <typename T, typename TG>
__global__ __launch_bounds__(256) void k_batch_reduce(BatchArg<T, TG> A, int G, int nsum) {
  __shared__ double sh[256];
  __shared__ double runs[2][256];
  const PassArg<T, TG> &D = A.d[blockIdx.x];
  const int64_t waves = grid_blocks(D.pl, G) * WAVES_PER_BLOCK;
  int64_t nb = (waves + 1023) / 1024;
  if (nb > 256) nb = 256;
  int64_t run = waves;
  if (nb > 1) {
    run = (waves + nb - 1) / nb;
    nb = (waves + run - 1) / run;
  } else {
    nb = 1;
  }
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t w0 = b * run, w1 = (w0 + run) < waves ? (w0 + run) : waves;
    for (int c = 0; c < nsum; ++c) {
      double s = 0.0;
      for (int64_t w = w0 + threadIdx.x; w < w1; w += 256) s += D.wsum[w * nsum + c];
      sh[threadIdx.x] = s;
      __syncthreads();
      for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
      }
      if (threadIdx.x == 0) runs[c][b] = sh[0];
      __syncthreads();
    }
  }
  for (int c = 0; c < nsum; ++c) {
    if (nb == 1) {
      if (threadIdx.x == 0) D.result[c] = runs[c][0];
      continue;
    }
    sh[threadIdx.x] = (int64_t)threadIdx.x < nb ? runs[c][threadIdx.x] : 0.0;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) D.result[c] = sh[0];
    __syncthreads();
  }
}

template <typename TG>
int width_class(int width) {
  const GC gc = pick_gc(width, VT<TG>::V);
  return gc.G * 16 + gc.C;
}

template <typename T, typename TG>
hipError_t launch_batch(const PassArg<T, TG> *d, int nd, int mode, hipStream_t s) {
  constexpr int V = VT<TG>::V;
  if (nd < 1 || nd > BATCH_MAX) return hipErrorInvalidValue;
  const GC gc = pick_gc(d[0].width, V);
  BatchArg<T, TG> A;
  A.nd = nd;
  A.b0[0] = 0;
  for (int i = 0; i < nd; ++i) {
    if (d[i].width > max_width<T>() || width_class<TG>(d[i].width) != gc.G * 16 + gc.C)
      return hipErrorInvalidValue;
    if (mode != 1 && d[i].pl.n_pieces * partial_row_bytes<T, TG>(gc) > d[i].partial_bytes)
      return hipErrorInvalidValue;
    A.d[i] = d[i];
    A.b0[i + 1] = A.b0[i] + (grid_blocks(d[i].pl, gc.G) + 7) / 8 * 8;
  }
  for (int i = nd + 1; i <= BATCH_MAX; ++i) A.b0[i] = A.b0[nd];
  const dim3 grid((unsigned)A.b0[nd]);
  BMG_DISPATCH_GC(gc, {
    if (mode == 0)
      hipLaunchKernelGGL((k_batch<T, TG, GG, CC, 0>), grid, dim3(256), 0, s, A);
    else if (mode == 1)
      hipLaunchKernelGGL((k_batch<T, TG, GG, CC, 1>), grid, dim3(256), 0, s, A);
    else
      hipLaunchKernelGGL((k_batch<T, TG, GG, CC, 2>), grid, dim3(256), 0, s, A);
    for (int i = 0; i < nd; ++i) {
      const PassArg<T, TG> &D = d[i];
      if (D.pl.n_long == 0 || mode == 1) continue;
      const int64_t thr = D.pl.n_long * GG;
      if (mode == 0)
        hipLaunchKernelGGL((k_grad_fix<T, TG, GG, CC>), dim3((unsigned)((thr + 255) / 256)),
                           dim3(256), 0, s, D.pl, (const T *)D.partial, D.X, D.ldx, D.width, D.lam,
                           D.out, D.ldo);
      else
        hipLaunchKernelGGL((k_spmm_fix<T, TG, GG, CC, false>), dim3((unsigned)((thr + 255) / 256)),
                           dim3(256), 0, s, D.pl, (const T *)D.partial, D.coef, D.X, D.ldx, D.kx,
                           D.M, D.ldm, D.width, D.out, D.ldo);
    }
  });
  if (mode != 2)
    hipLaunchKernelGGL((k_batch_reduce<T, TG>), dim3((unsigned)nd), dim3(256), 0, s, A, gc.G,
                       mode == 0 ? 1 : 2);
  return hipGetLastError();
}

}  // namespace bmg
