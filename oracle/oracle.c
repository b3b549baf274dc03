/*
 * CPU oracle: sparse loops of BM-Global for matrix completion, plain FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the GPU
 * library and never calls it.
 *
 * Omega is given in CSR form: row_ptr[m+1] (int64), col[nnz] (int32, sorted
 * within a row), values val[nnz] (float64).  Dense factors are row-major with
 * a leading dimension.  Every loop is the plain definition; rows are
 * independent, so the row loops may run on several threads without changing a
 * single bit of the result.
 */
#include <stdint.h>
#include <stddef.h>

/* Omega-sampled residual (the gradient of the MC loss is sparse and equals
 * P_Omega(X - A); problem (MC) and its MF form, Section 1):
 *   R[p] = sum_r X[i,r] Y[j,r] - A[p]  for every stored entry p = (i, j).
 * If A is NULL the values are taken as zero, which gives P_Omega(X Y^T). */
void orc_sddmm(int64_t m, const int64_t *row_ptr, const int32_t *col, const double *A, int k,
               const double *X, int64_t ldx, const double *Y, int64_t ldy, double *R) {
#pragma omp parallel for schedule(dynamic, 32) if (row_ptr[m] > 200000)
  for (int64_t i = 0; i < m; i++) {
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; p++) {
      int64_t j = col[p];
      double s = 0.0;
      for (int r = 0; r < k; r++) s += X[i * ldx + r] * Y[j * ldy + r];
      R[p] = s - (A ? A[p] : 0.0);
    }
  }
}

/* Sparse times dense, row orientation: C[i,:] = sum_{p in row i} S[p] * B[col[p],:]
 * (C is m x q, overwritten). */
void orc_spmm(int64_t m, const int64_t *row_ptr, const int32_t *col, const double *S, int q,
              const double *B, int64_t ldb, double *C, int64_t ldc) {
#pragma omp parallel for schedule(dynamic, 32) if (row_ptr[m] > 200000)
  for (int64_t i = 0; i < m; i++) {
    for (int c = 0; c < q; c++) C[i * ldc + c] = 0.0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; p++) {
      const double *b = B + (int64_t)col[p] * ldb;
      for (int c = 0; c < q; c++) C[i * ldc + c] += S[p] * b[c];
    }
  }
}

/* Transposed product: C[j,:] = sum_{p : col[p] = j} S[p] * B[row(p),:]
 * (C is n x q, overwritten).  One thread walks Omega in CSR order, so the
 * summation order for every output row is by increasing row index. */
void orc_spmm_t(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *S,
                int q, const double *B, int64_t ldb, double *C, int64_t ldc) {
  for (int64_t j = 0; j < n; j++)
    for (int c = 0; c < q; c++) C[j * ldc + c] = 0.0;
  for (int64_t i = 0; i < m; i++) {
    const double *b = B + i * ldb;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; p++) {
      double *o = C + (int64_t)col[p] * ldc;
      for (int c = 0; c < q; c++) o[c] += S[p] * b[c];
    }
  }
}

/* Sum of squares in index order, one partial per row, rows added in order. */
double orc_sumsq_rows(int64_t m, const int64_t *row_ptr, const double *R) {
  double tot = 0.0;
  for (int64_t i = 0; i < m; i++) {
    double s = 0.0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; p++) s += R[p] * R[p];
    tot += s;
  }
  return tot;
}
