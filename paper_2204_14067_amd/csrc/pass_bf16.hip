// Sparse-pass launchers instantiated for FP32 factors, BF16 gathers.
#include "rowpass.h"

namespace bmg {
#define BMG_INST_PASS(T, TG)                                                                    \
  template hipError_t launch_grad<T, TG>(const Plan &, const T *, const T *, int, const TG *, int,   \
                                         int, double, T *, int, PassScratch, int64_t *,              \
                                         hipStream_t);                                               \
  template hipError_t launch_sddmm<T, TG>(const Plan &, const T *, const T *, int, const TG *, int,  \
                                          int, T *, PassScratch, hipStream_t);                       \
  template hipError_t launch_spmm<T, TG>(const Plan &, const T *, const TG *, int, int, double,      \
                                         const T *, int, int, const T *, int, T *, int, PassScratch, \
                                         hipStream_t);
BMG_INST_PASS(float, bf16_t)
template hipError_t launch_batch<float, bf16_t>(const PassArg<float, bf16_t> *, int, int, hipStream_t);
template int width_class<bf16_t>(int);
}  // namespace bmg
