// Small dense FP64 linear algebra on the host (declarations).
#pragma once

namespace bmg {
// ---------------------------------------------------------------- small FP64 linear algebra (host)
namespace la {
// Symmetric eigen-decomposition A = V diag(w) V^T, w descending.  A: n x n
// row-major (only read).  V may be null (values only).
void sym_eig(int n, const double *A, double *w, double *V);
// Pivoted Cholesky of a PSD matrix with a relative cut: P^T G P ~ R^T R with R
// upper-trapezoidal r x n; stops when the largest remaining diagonal is
// <= tol * (largest initial diagonal).  perm[n] receives the pivot order.
int chol_pivoted(int n, const double *G, double tol, int *perm, double *R);
// Plain Cholesky G = R^T R (R upper, row-major n x n).  false if not PD.
bool chol(int n, const double *G, double *R);
// Inverse of an upper-triangular matrix (n x n row-major) into Rinv.
void tri_inv_upper(int n, const double *R, double *Rinv);
// Inverse of an SPD matrix via Cholesky; false if not PD.
bool spd_inv(int n, const double *A, double *Ainv);
}  // namespace la
}  // namespace bmg
