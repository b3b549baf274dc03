// Work units of a load-balancing plan for one-wave-per-unit kernels: unit
// u < n_short is a short row, unit n_short + p is piece p of a long row.
#pragma once
#include <hip/hip_runtime.h>

#include "bmg_internal.h"

namespace bmg {

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

}  // namespace bmg
