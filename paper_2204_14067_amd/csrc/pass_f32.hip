// Sparse-pass launchers instantiated for FP32 factors, FP32 gathers.
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
BMG_INST_PASS(float, float)
template hipError_t launch_batch<float, float>(const PassArg<float, float> *, int, int, hipStream_t);
template int width_class<float>(int);
}  // namespace bmg
