// Small dense FP64 linear algebra for the q x q steps of the prox
// (Rayleigh-Ritz eigenvalues, the exact SVD of the projected matrix through
// its Gram matrix, orthonormalisation by pivoted Cholesky, the Nystrom core of
// the initialisation and the k x k preconditioner of the BM step).
//
// Symmetric eigenproblem: Householder reduction to tridiagonal form followed
// by implicit symmetric QR steps with the Wilkinson shift (Golub & Van Loan,
// Matrix Computations, Secs. 8.3.1-8.3.3), eigenvectors accumulated from the
// reflectors and Givens rotations.  Row-major storage throughout.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "linalg.h"

namespace bmg {
namespace la {

static inline double &at(std::vector<double> &A, int n, int i, int j) { return A[(size_t)i * n + j]; }

void sym_eig(int n, const double *A0, double *w, double *Vout) {
  if (n <= 0) return;
  std::vector<double> A(A0, A0 + (size_t)n * n);
  // symmetrise against rounding in the input
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double s = 0.5 * (at(A, n, i, j) + at(A, n, j, i));
      at(A, n, i, j) = at(A, n, j, i) = s;
    }
  const bool vec = Vout != nullptr;
  std::vector<double> Q;
  if (vec) {
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) at(Q, n, i, i) = 1.0;
  }
  std::vector<double> v(n), p(n);
  // --- Householder tridiagonalisation: A <- H A H, Q <- Q H with
  // H = I - 2 v v^T / (v^T v) acting on indices k+1 .. n-1.
  for (int k = 0; k + 2 < n; ++k) {
    double sig = 0.0;
    for (int i = k + 1; i < n; ++i) sig += at(A, n, i, k) * at(A, n, i, k);
    double tail = sig - at(A, n, k + 1, k) * at(A, n, k + 1, k);
    if (tail <= 0.0) continue;  // column already tridiagonal
    sig = sqrt(sig);
    const double x0 = at(A, n, k + 1, k);
    const double alpha = x0 >= 0 ? -sig : sig;
    for (int i = k + 1; i < n; ++i) v[i] = at(A, n, i, k);
    v[k + 1] -= alpha;
    double beta = 0.0;
    for (int i = k + 1; i < n; ++i) beta += v[i] * v[i];
    if (beta == 0.0) continue;
    const double tau = 2.0 / beta;
    // left: rows k+1.. of A: A -= tau v (v^T A)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += v[i] * at(A, n, i, j);
      p[j] = tau * s;
    }
    for (int i = k + 1; i < n; ++i)
      for (int j = 0; j < n; ++j) at(A, n, i, j) -= v[i] * p[j];
    // right: columns k+1.. of A: A -= tau (A v) v^T
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += at(A, n, i, j) * v[j];
      p[i] = tau * s;
    }
    for (int i = 0; i < n; ++i)
      for (int j = k + 1; j < n; ++j) at(A, n, i, j) -= p[i] * v[j];
    if (vec) {
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = k + 1; j < n; ++j) s += at(Q, n, i, j) * v[j];
        p[i] = tau * s;
      }
      for (int i = 0; i < n; ++i)
        for (int j = k + 1; j < n; ++j) at(Q, n, i, j) -= p[i] * v[j];
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = at(A, n, i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = 0.5 * (at(A, n, i, i + 1) + at(A, n, i + 1, i));
  // --- implicit symmetric QR with Wilkinson shift on the tridiagonal (d, e)
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int guard = 0;
  while (hi > 0 && guard < 60 * n) {
    // deflate from the bottom
    if (fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi])) || e[hi - 1] == 0.0) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && !(fabs(e[lo - 1]) <= eps * (fabs(d[lo - 1]) + fabs(d[lo])))) --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    ++guard;
    // Wilkinson shift from the trailing 2x2 of the block [lo, hi]
    const double delta = 0.5 * (d[hi - 1] - d[hi]);
    const double es = e[hi - 1] * e[hi - 1];
    const double den = delta + copysign(sqrt(delta * delta + es), delta == 0.0 ? 1.0 : delta);
    const double mu = d[hi] - es / den;
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) { c = x / r; s = -z / r; }
      if (k > lo) e[k - 1] = r;
      const double a = d[k], b = e[k], cc = d[k + 1];
      d[k] = c * c * a - 2.0 * c * s * b + s * s * cc;
      d[k + 1] = s * s * a + 2.0 * c * s * b + c * c * cc;
      e[k] = c * s * (a - cc) + (c * c - s * s) * b;
      if (k + 1 < hi) {
        x = e[k];
        z = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      if (vec) {
        for (int i = 0; i < n; ++i) {
          const double qk = at(Q, n, i, k), qk1 = at(Q, n, i, k + 1);
          at(Q, n, i, k) = c * qk - s * qk1;
          at(Q, n, i, k + 1) = s * qk + c * qk1;
        }
      }
    }
  }
  // sort descending
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] > d[b]; });
  for (int i = 0; i < n; ++i) w[i] = d[ord[i]];
  if (vec)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) Vout[(size_t)i * n + j] = at(Q, n, i, ord[j]);
}

int chol_pivoted(int n, const double *G, double tol, int *perm, double *R) {
  std::vector<double> A(G, G + (size_t)n * n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  memset(R, 0, sizeof(double) * (size_t)n * n);
  double dmax0 = 0.0;
  for (int i = 0; i < n; ++i) dmax0 = std::max(dmax0, A[(size_t)i * n + i]);
  if (dmax0 <= 0.0) return 0;
  // A holds the Schur complement in the permuted order; R rows are built in order.
  int r = 0;
  for (int j = 0; j < n; ++j) {
    int piv = j;
    double best = A[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i)
      if (A[(size_t)i * n + i] > best) { best = A[(size_t)i * n + i]; piv = i; }
    if (!(best > tol * dmax0)) break;
    if (piv != j) {  // symmetric swap of rows/cols j and piv, and of R's columns
      for (int i = 0; i < n; ++i) std::swap(A[(size_t)j * n + i], A[(size_t)piv * n + i]);
      for (int i = 0; i < n; ++i) std::swap(A[(size_t)i * n + j], A[(size_t)i * n + piv]);
      for (int i = 0; i < j; ++i) std::swap(R[(size_t)i * n + j], R[(size_t)i * n + piv]);
      std::swap(perm[j], perm[piv]);
    }
    const double rjj = sqrt(A[(size_t)j * n + j]);
    R[(size_t)j * n + j] = rjj;
    for (int i = j + 1; i < n; ++i) R[(size_t)j * n + i] = A[(size_t)j * n + i] / rjj;
    for (int i = j + 1; i < n; ++i)
      for (int l = j + 1; l < n; ++l)
        A[(size_t)i * n + l] -= R[(size_t)j * n + i] * R[(size_t)j * n + l];
    r = j + 1;
  }
  return r;
}

bool chol(int n, const double *G, double *R) {
  memset(R, 0, sizeof(double) * (size_t)n * n);
  for (int j = 0; j < n; ++j) {
    double s = G[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= R[(size_t)k * n + j] * R[(size_t)k * n + j];
    if (!(s > 0.0)) return false;
    const double rjj = sqrt(s);
    R[(size_t)j * n + j] = rjj;
    for (int i = j + 1; i < n; ++i) {
      double t = G[(size_t)j * n + i];
      for (int k = 0; k < j; ++k) t -= R[(size_t)k * n + j] * R[(size_t)k * n + i];
      R[(size_t)j * n + i] = t / rjj;
    }
  }
  return true;
}

void tri_inv_upper(int n, const double *R, double *X) {
  // solve R X = I column by column (back substitution)
  memset(X, 0, sizeof(double) * (size_t)n * n);
  for (int c = 0; c < n; ++c) {
    for (int i = c; i >= 0; --i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = i + 1; k <= c; ++k) s -= R[(size_t)i * n + k] * X[(size_t)k * n + c];
      X[(size_t)i * n + c] = s / R[(size_t)i * n + i];
    }
  }
}

bool spd_inv(int n, const double *A, double *Ainv) {
  std::vector<double> R((size_t)n * n), Ri((size_t)n * n);
  if (!chol(n, A, R.data())) return false;
  tri_inv_upper(n, R.data(), Ri.data());
  // A^{-1} = R^{-1} R^{-T}
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = std::max(i, j); k < n; ++k) s += Ri[(size_t)i * n + k] * Ri[(size_t)j * n + k];
      Ainv[(size_t)i * n + j] = s;
    }
  return true;
}

}  // namespace la
}  // namespace bmg
