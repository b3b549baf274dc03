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

// Built twice (baseline x86-64 and x86-64-v3 with AVX2/FMA) into namespaces
// bmg::la_generic and bmg::la_v3; linalg_dispatch.cpp picks one at run time.
#ifndef LA_IMPL
#error "compile with -DLA_IMPL=la_generic or -DLA_IMPL=la_v3"
#endif

namespace bmg {
namespace LA_IMPL {

static inline double &at(std::vector<double> &A, int n, int i, int j) { return A[(size_t)i * n + j]; }

// a . b with eight independent partial sums added in a fixed order (the
// compiler can keep them in vector registers; a single running sum is one
// long dependency chain).  Deterministic for given inputs.
static inline double dot(const double *a, const double *b, int n) {
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int i = 0;
  for (; i + 8 <= n; i += 8)
    for (int l = 0; l < 8; ++l) s[l] += a[i + l] * b[i + l];
  for (int l = 0; i < n; ++i, ++l) s[l] += a[i] * b[i];
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

void sym_eig(int n, const double *A0, double *w, double *Vout) {
  if (n <= 0) return;
  // Only the lower triangle is kept and updated (j <= i); it starts as the
  // mean of A0 and A0^T against rounding asymmetry in the input.
  std::vector<double> A((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) at(A, n, i, j) = 0.5 * (A0[(size_t)i * n + j] + A0[(size_t)j * n + i]);
  const bool vec = Vout != nullptr;
  // --- Householder tridiagonalisation.  Step k reflects rows/columns k+1..n-1
  // with H = I - tau v v^T; the trailing block gets the symmetric rank-2 update
  // A22 <- A22 - v w^T - w v^T,  w = p - (tau/2)(p^T v) v,  p = tau A22 v.
  // p is formed from the lower triangle row by row: row i contributes its
  // dot product with v to p_i and its entries times v_i to p_j, j < i.
  std::vector<double> vs((size_t)n * n, 0.0), taus(n, 0.0), p(n), wv(n);
  std::vector<double> d(n), e(n, 0.0);
  for (int k = 0; k + 2 < n; ++k) {
    double *v = &vs[(size_t)k * n];
    double sig = 0.0;
    for (int i = k + 1; i < n; ++i) sig += at(A, n, i, k) * at(A, n, i, k);
    const double x0 = at(A, n, k + 1, k);
    if (sig - x0 * x0 <= 0.0) continue;  // already tridiagonal in this column
    const double nrm = sqrt(sig);
    const double alpha = x0 >= 0 ? -nrm : nrm;
    for (int i = k + 1; i < n; ++i) v[i] = at(A, n, i, k);
    v[k + 1] -= alpha;
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double tau = 2.0 / vv;
    taus[k] = tau;
    for (int i = k + 1; i < n; ++i) p[i] = 0.0;
    for (int i = k + 1; i < n; ++i) {
      // one pass over row i's part left of the diagonal: its dot product with
      // v (eight partial sums, added in a fixed order) and its entries times v_i
      const double *row = &A[(size_t)i * n];
      const double vi = v[i];
      double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      int j = k + 1;
      for (; j + 8 <= i; j += 8)
        for (int l = 0; l < 8; ++l) {
          a[l] += row[j + l] * v[j + l];
          p[j + l] += row[j + l] * vi;
        }
      for (int l = 0; j < i; ++j, ++l) {
        a[l] += row[j] * v[j];
        p[j] += row[j] * vi;
      }
      p[i] += (((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]))) + row[i] * vi;
    }
    for (int i = k + 1; i < n; ++i) p[i] *= tau;
    double pv = 0.0;
    for (int i = k + 1; i < n; ++i) pv += p[i] * v[i];
    for (int i = k + 1; i < n; ++i) wv[i] = p[i] - 0.5 * tau * pv * v[i];
    for (int i = k + 1; i < n; ++i) {
      double *row = &A[(size_t)i * n];
      const double vi = v[i], wi = wv[i];
      for (int j = k + 1; j <= i; ++j) row[j] -= vi * wv[j] + wi * v[j];
    }
    at(A, n, k + 1, k) = alpha;
    for (int i = k + 2; i < n; ++i) at(A, n, i, k) = 0.0;
  }
  for (int i = 0; i < n; ++i) d[i] = at(A, n, i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = at(A, n, i + 1, i);
  // Z = Q^T with Q = H_0 H_1 ... H_{n-3}, accumulated backwards on rows
  std::vector<double> Z;
  if (vec) {
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    // Q = H_0 (H_1 (... H_{n-3})); Z = Q^T = (... H_{n-3}) ... H_0 applied from the right:
    // build Q column-block-wise: Q[k+1:, k+1:] = H_k Q[k+1:, k+1:]  (k descending),
    // kept as Z (rows of Z are columns of Q).
    for (int k = n - 3; k >= 0; --k) {
      if (taus[k] == 0.0) continue;
      const double *v = &vs[(size_t)k * n];
      const double tau = taus[k];
      // for each column c >= k+1 of Q (row c of Z): q_c[k+1:] -= tau v (v^T q_c[k+1:])
      for (int c = k + 1; c < n; ++c) {
        double *zc = &Z[(size_t)c * n];
        const double acc = tau * dot(v + k + 1, zc + k + 1, n - k - 1);
        for (int i = k + 1; i < n; ++i) zc[i] -= acc * v[i];
      }
    }
  }
  // --- implicit symmetric QR with Wilkinson shift on the tridiagonal (d, e);
  // rotations of columns k, k+1 of Q are rotations of rows k, k+1 of Z
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int guard = 0;
  while (hi > 0 && guard < 60 * n) {
    if (fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi])) || e[hi - 1] == 0.0) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && !(fabs(e[lo - 1]) <= eps * (fabs(d[lo - 1]) + fabs(d[lo])))) --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    ++guard;
    const double delta = 0.5 * (d[hi - 1] - d[hi]);
    const double es = e[hi - 1] * e[hi - 1];
    const double den = delta + copysign(sqrt(delta * delta + es), delta == 0.0 ? 1.0 : delta);
    const double mu = d[hi] - es / den;
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = sqrt(x * x + z * z);   // Gram-matrix entries: no overflow risk
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
        double *zk = &Z[(size_t)k * n], *zk1 = &Z[(size_t)(k + 1) * n];
        for (int i = 0; i < n; ++i) {
          const double qk = zk[i], qk1 = zk1[i];
          zk[i] = c * qk - s * qk1;
          zk1[i] = s * qk + c * qk1;
        }
      }
    }
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] > d[b]; });
  for (int i = 0; i < n; ++i) w[i] = d[ord[i]];
  if (vec)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) Vout[(size_t)i * n + j] = Z[(size_t)ord[j] * n + i];
}

int chol_pivoted(int n, const double *G, double tol, int *perm, double *R) {
  // Left-looking with diagonal pivoting: dg holds the diagonal of the current
  // Schur complement (in pivot-position order); step j picks the largest,
  // swaps positions j and piv (perm and the columns of the rows of R already
  // built), and forms row j of R from G and the rows above it:
  //   R_jc = (G_{perm j, perm c} - sum_{l<j} R_lj R_lc) / R_jj,  c > j.
  // Only the rows of R already built are read: n^3/3 flops in all.
  for (int i = 0; i < n; ++i) perm[i] = i;
  memset(R, 0, sizeof(double) * (size_t)n * n);
  std::vector<double> dg(n), acc(n);
  double dmax0 = 0.0;
  for (int i = 0; i < n; ++i) {
    dg[i] = G[(size_t)i * n + i];
    dmax0 = std::max(dmax0, dg[i]);
  }
  if (dmax0 <= 0.0) return 0;
  int r = 0;
  for (int j = 0; j < n; ++j) {
    int piv = j;
    double best = dg[j];
    for (int i = j + 1; i < n; ++i)
      if (dg[i] > best) { best = dg[i]; piv = i; }
    if (!(best > tol * dmax0)) break;
    if (piv != j) {
      std::swap(dg[j], dg[piv]);
      std::swap(perm[j], perm[piv]);
      for (int l = 0; l < j; ++l) std::swap(R[(size_t)l * n + j], R[(size_t)l * n + piv]);
    }
    const double rjj = sqrt(dg[j]);
    double *rj = &R[(size_t)j * n];
    rj[j] = rjj;
    const double *g = &G[(size_t)perm[j] * n];
    for (int c = j + 1; c < n; ++c) acc[c] = g[perm[c]];
    for (int l = 0; l < j; ++l) {
      const double *rl = &R[(size_t)l * n];
      const double f = rl[j];
      for (int c = j + 1; c < n; ++c) acc[c] -= f * rl[c];
    }
    const double inv = 1.0 / rjj;
    for (int c = j + 1; c < n; ++c) {
      rj[c] = acc[c] * inv;
      dg[c] -= rj[c] * rj[c];
    }
    r = j + 1;
  }
  return r;
}

bool chol(int n, const double *G, double *R) {
  // right-looking: row j of R from the current Schur complement (upper
  // triangle only, kept in R itself), then a rank-1 update of the trailing rows
  memset(R, 0, sizeof(double) * (size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int l = i; l < n; ++l) R[(size_t)i * n + l] = G[(size_t)i * n + l];
  for (int j = 0; j < n; ++j) {
    double *rj = &R[(size_t)j * n];
    const double s = rj[j];
    if (!(s > 0.0)) return false;
    const double rjj = sqrt(s), inv = 1.0 / rjj;
    rj[j] = rjj;
    for (int l = j + 1; l < n; ++l) rj[l] *= inv;
    for (int i = j + 1; i < n; ++i) {
      double *ri = &R[(size_t)i * n];
      const double f = rj[i];
      for (int l = i; l < n; ++l) ri[l] -= f * rj[l];
    }
  }
  return true;
}

void tri_inv_upper(int n, const double *R, double *X) {
  // rows from the bottom, four at a time: X[i, :] = (e_i - sum_{k > i} R[i, k]
  // X[k, :]) / R[i, i].  The rows below the block are final; each of them is
  // loaded once for the four rows of the block (row k of X is zero left of
  // column k, so every update is a contiguous axpy), then the block's own
  // rows are finished bottom-up.
  memset(X, 0, sizeof(double) * (size_t)n * n);
  int i1 = n;
  while (i1 > 0) {
    const int nb = std::min(4, i1), i0 = i1 - nb;
    double *x0 = &X[(size_t)i0 * n];
    for (int r = 0; r < nb; ++r) x0[(size_t)r * n + i0 + r] = 1.0;
    for (int k = i1; k < n; ++k) {
      const double *xk = &X[(size_t)k * n];
      double f[4] = {0, 0, 0, 0};
      for (int r = 0; r < nb; ++r) f[r] = R[(size_t)(i0 + r) * n + k];
      if (nb == 4) {
        double *a = x0, *b = x0 + n, *c = x0 + 2 * (size_t)n, *d = x0 + 3 * (size_t)n;
        for (int col = k; col < n; ++col) {
          const double v = xk[col];
          a[col] -= f[0] * v;
          b[col] -= f[1] * v;
          c[col] -= f[2] * v;
          d[col] -= f[3] * v;
        }
      } else {
        for (int r = 0; r < nb; ++r) {
          double *xr = x0 + (size_t)r * n;
          for (int col = k; col < n; ++col) xr[col] -= f[r] * xk[col];
        }
      }
    }
    for (int i = i1 - 1; i >= i0; --i) {
      double *xi = &X[(size_t)i * n];
      const double *ri = &R[(size_t)i * n];
      for (int k = i + 1; k < i1; ++k) {
        const double f = ri[k];
        const double *xk = &X[(size_t)k * n];
        for (int col = k; col < n; ++col) xi[col] -= f * xk[col];
      }
      const double inv = 1.0 / ri[i];
      for (int col = i; col < n; ++col) xi[col] *= inv;
    }
    i1 = i0;
  }
}

bool spd_inv(int n, const double *A, double *Ainv) {
  std::vector<double> R((size_t)n * n), Ri((size_t)n * n);
  if (!chol(n, A, R.data())) return false;
  tri_inv_upper(n, R.data(), Ri.data());
  // A^{-1} = R^{-1} R^{-T}: entry (i, j) is the dot of rows i and j of R^{-1}
  // from column max(i, j) on (the rows are zero left of their diagonal)
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      const double s = dot(&Ri[(size_t)i * n + j], &Ri[(size_t)j * n + j], n - j);
      Ainv[(size_t)i * n + j] = s;
      Ainv[(size_t)j * n + i] = s;
    }
  return true;
}

}  // namespace LA_IMPL
}  // namespace bmg
