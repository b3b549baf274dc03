// bmg_sddmm_static: the sampled residual of bmg_sddmm straight from a device
// CSR, for callers that cannot allocate device memory.  Its only scratch (the
// per-wave partial sums of 1/2 sum R^2, the two-stage reduction's first-stage
// sums and results, and the CSR check's flag word) is the file-scope device
// array `scratch` below; host code reaches it only through the per-device
// address that hipGetSymbolAddress returns.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>
#include <string>

#include "bmg.h"
#include "bmg_internal.h"

using namespace bmg;

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)BMG_STATIC_SCRATCH_BYTES;
// scratch layout (bytes): flag word | first-stage sums (256 x 2) | result (2) | per-wave pairs
constexpr size_t OFF_FLAG = 0, OFF_WPART = 256, OFF_RESULT = OFF_WPART + 256 * 2 * 8,
                 OFF_WSUM = OFF_RESULT + 256;
constexpr int64_t WSUM_PAIRS = (int64_t)((SCRATCH_BYTES - OFF_WSUM) / 16);
// A sampled-residual grid over rows in their own order has one wave per 64 / TL
// rows (TL = 8 or 16 lanes per row, so at least 4 rows per wave), rounded up to
// whole blocks of 4 waves: at most m / 4 + 4 waves.
constexpr int64_t MAX_ROWS = 4 * (WSUM_PAIRS - 4);
static_assert(MAX_ROWS == BMG_STATIC_MAX_ROWS, "bmg.h states the row limit of the static scratch");

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// flag bits: 1 row_ptr[0] != 0 or row_ptr[m] != nnz, 2 a row range outside [0, nnz]
// or decreasing, 4 column index outside [0, n), 8 columns not strictly
// increasing within a row, 16 non-finite value
__global__ void k_static_clear(int *flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) flag[0] = 0;
}
// One wave per row (grid-stride over rows): every entry read lies in [0, nnz)
// because the row's range is checked first.
__global__ __launch_bounds__(256) void k_static_check(int64_t m, int64_t n, int64_t nnz,
                                                      const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val, int *flag) {
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  if (wave0 == 0 && lane == 0 && (row_ptr[0] != 0 || row_ptr[m] != nnz)) atomicOr(flag, 1);
  for (int64_t i = wave0; i < m; i += nwaves) {
    const int64_t beg = row_ptr[i], end = row_ptr[i + 1];
    if (beg < 0 || end > nnz || end < beg) {
      if (lane == 0) atomicOr(flag, 2);
      continue;
    }
    int bits = 0;
    for (int64_t p = beg + lane; p < end; p += 64) {
      const int c = col[p];
      if (c < 0 || (int64_t)c >= n) bits |= 4;
      if (p > beg && c <= col[p - 1]) bits |= 8;
      if (!isfinite(val[p])) bits |= 16;
    }
    if (bits) atomicOr(flag, bits);
  }
}

static bmg_status sfail(bmg_status st, const std::string &msg) { return set_error(st, msg); }

extern "C" bmg_status bmg_sddmm_static(const bmg_csr *csr, const double *W, const double *H, int k,
                                       int ld, double *R, double *half_sq, void *stream) {
  // argument checks come before any HIP call
  if (!csr) return sfail(BMG_EINVAL, "bmg_sddmm_static: null CSR");
  const int64_t m = csr->m, n = csr->n, nnz = csr->nnz;
  if (m < 0 || n < 0 || nnz < 0 || nnz > (int64_t)INT32_MAX || n > (int64_t)INT32_MAX)
    return sfail(BMG_EINVAL, "bmg_sddmm_static: bad shape");
  if (m > MAX_ROWS)
    return sfail(BMG_ENOMEM, "bmg_sddmm_static: " + std::to_string(m) +
                                 " rows exceed the static scratch (at most " +
                                 std::to_string(MAX_ROWS) + " rows per call)");
  if (k < 0 || k > max_width<double>() || ld < k || ld % 8 != 0)
    return sfail(BMG_EINVAL, "bmg_sddmm_static: bad k / ld");
  if (k > 0 && (!W || !H)) return sfail(BMG_EINVAL, "bmg_sddmm_static: null factor");
  if ((((uintptr_t)W) & 15) || (((uintptr_t)H) & 15))
    return sfail(BMG_EINVAL, "bmg_sddmm_static: factors not 16-byte aligned");
  if (m > 0 && !csr->row_ptr) return sfail(BMG_EINVAL, "bmg_sddmm_static: null row_ptr");
  if (nnz > 0 && (!csr->col || !csr->val)) return sfail(BMG_EINVAL, "bmg_sddmm_static: null CSR array");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
    return sfail(BMG_EDEVICE, "bmg_sddmm_static: no current device");
  unsigned char *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
      void *p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return sfail(BMG_EDEVICE, std::string("bmg_sddmm_static: hipGetSymbolAddress: ") +
                                      hipGetErrorString(e));
      g_ptr[dev] = p;
    }
    base = (unsigned char *)g_ptr[dev];
  }
  int *flag = (int *)(base + OFF_FLAG);
  double *wpart = (double *)(base + OFF_WPART), *result = (double *)(base + OFF_RESULT),
         *wsum = (double *)(base + OFF_WSUM);
  double h = 0.0;
  if (m > 0) {
    int hf = 0;
    hipLaunchKernelGGL(k_static_clear, dim3(1), dim3(64), 0, s, flag);
    const int64_t nb = std::min<int64_t>((m + 3) / 4, 4096);
    hipLaunchKernelGGL(k_static_check, dim3((unsigned)nb), dim3(256), 0, s, m, n, nnz,
                       csr->row_ptr, csr->col, csr->val, flag);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return sfail(BMG_EDEVICE, std::string("bmg_sddmm_static: ") + hipGetErrorString(e));
    if (hf & 1) return sfail(BMG_EINVAL, "bmg_sddmm_static: row_ptr[0] != 0 or row_ptr[m] != nnz");
    if (hf & 2) return sfail(BMG_EINVAL, "bmg_sddmm_static: row_ptr decreases or leaves [0, nnz]");
    if (hf & 4) return sfail(BMG_EINVAL, "bmg_sddmm_static: column index out of range");
    if (hf & 8) return sfail(BMG_EINVAL, "bmg_sddmm_static: columns not strictly increasing within a row");
    if (hf & 16) return sfail(BMG_ENONFINITE, "bmg_sddmm_static: non-finite observed value");
  }
  if (nnz > 0) {
    Plan pl;
    pl.nrows = m;
    pl.ncols = n;
    pl.nnz = nnz;
    pl.ptr = csr->row_ptr;
    pl.idx = csr->col;
    pl.short_rows = nullptr;  // rows in their own order
    pl.n_short = m;
    PassScratch sc;
    sc.wsum = wsum;
    sc.wpart = wpart;
    sc.result = result;
    sc.partial = nullptr;     // no long-row pieces
    sc.partial_bytes = 0;
    hipError_t e = launch_sddmm<double, double>(pl, csr->val, W, ld, H, ld, k, R, sc, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, result, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return sfail(BMG_EDEVICE, std::string("bmg_sddmm_static: ") + hipGetErrorString(e));
  }
  if (half_sq) *half_sq = 0.5 * h;
  return BMG_OK;
}
