// Run-time choice between the two builds of linalg.cpp: the x86-64-v3 one
// (AVX2 + FMA) when the host CPU has both, else the baseline one.
#include "linalg.h"

namespace bmg {
#define BMG_LA_DECLS                                                            \
  void sym_eig(int n, const double *A, double *w, double *V);                  \
  int chol_pivoted(int n, const double *G, double tol, int *perm, double *R);  \
  bool chol(int n, const double *G, double *R);                                 \
  void tri_inv_upper(int n, const double *R, double *Rinv);                     \
  bool spd_inv(int n, const double *A, double *Ainv);
namespace la_generic { BMG_LA_DECLS }
namespace la_v3 { BMG_LA_DECLS }
#undef BMG_LA_DECLS

namespace la {
static bool use_v3() {
  static const bool v = [] {
    __builtin_cpu_init();
    return __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
  }();
  return v;
}
void sym_eig(int n, const double *A, double *w, double *V) {
  if (use_v3()) la_v3::sym_eig(n, A, w, V);
  else la_generic::sym_eig(n, A, w, V);
}
int chol_pivoted(int n, const double *G, double tol, int *perm, double *R) {
  return use_v3() ? la_v3::chol_pivoted(n, G, tol, perm, R)
                  : la_generic::chol_pivoted(n, G, tol, perm, R);
}
bool chol(int n, const double *G, double *R) {
  return use_v3() ? la_v3::chol(n, G, R) : la_generic::chol(n, G, R);
}
void tri_inv_upper(int n, const double *R, double *Rinv) {
  if (use_v3()) la_v3::tri_inv_upper(n, R, Rinv);
  else la_generic::tri_inv_upper(n, R, Rinv);
}
bool spd_inv(int n, const double *A, double *Ainv) {
  return use_v3() ? la_v3::spd_inv(n, A, Ainv) : la_generic::spd_inv(n, A, Ainv);
}
}  // namespace la
}  // namespace bmg
