/*
 * Seeded synthetic matrix-completion inputs (sampling pattern Omega and the
 * observed values A_Omega).  Input generation only: nothing in this file
 * computes any step of the solver.  Both the CPU oracle and the GPU path read
 * the arrays it produces.
 *
 * Output layout (caller allocates, row-major CSR, sorted, duplicate-free):
 *   row_ptr[m+1] int64, col[nnz] int32, val[nnz] float64.
 *
 * Randomness: every row draws from its own xoshiro256** stream seeded by
 * SplitMix64(seed, stream id), so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------- RNG: SplitMix64 seeding + xoshiro256** (Blackman, Vigna) */
static inline uint64_t sm64(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
typedef struct { uint64_t s[4]; } rng_t;
static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static inline uint64_t rng_next(rng_t *r) {
  uint64_t *s = r->s;
  uint64_t res = rotl(s[1] * 5, 7) * 9, t = s[1] << 17;
  s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3]; s[2] ^= t; s[3] = rotl(s[3], 45);
  return res;
}
static void rng_init(rng_t *r, uint64_t seed, uint64_t stream) {
  uint64_t s = seed ^ (0xD1B54A32D192ED03ULL * (stream + 1));
  for (int i = 0; i < 4; i++) r->s[i] = sm64(&s);
}
/* uniform in (0,1) */
static inline double rng_u01(rng_t *r) { return ((rng_next(r) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
static inline uint64_t rng_below(rng_t *r, uint64_t n) { /* Lemire-free simple rejection */
  uint64_t lim = UINT64_MAX - UINT64_MAX % n, x;
  do { x = rng_next(r); } while (x >= lim);
  return x % n;
}
static inline double rng_normal(rng_t *r) { /* Box-Muller, one output */
  double u1 = rng_u01(r), u2 = rng_u01(r);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}
static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

/* ---------------------------------------------------------------- uniform Omega
 * nnz distinct linear indices drawn uniformly without replacement from [0, m*n)
 * (Floyd's algorithm with a hash set), then sorted into CSR order. */
typedef struct { int64_t *keys; int64_t cap; } hset_t;
static int hset_insert(hset_t *h, int64_t key) { /* 1 if newly inserted */
  uint64_t x = (uint64_t)key * 0x9E3779B97F4A7C15ULL;
  int64_t i = (int64_t)(x >> 17) & (h->cap - 1);
  while (h->keys[i] != -1) {
    if (h->keys[i] == key) return 0;
    i = (i + 1) & (h->cap - 1);
  }
  h->keys[i] = key;
  return 1;
}

int synth_uniform_pattern(int64_t m, int64_t n, int64_t nnz, uint64_t seed,
                          int64_t *row_ptr, int32_t *col) {
  int64_t total = m * n;
  if (nnz < 0 || nnz > total) return -1;
  int64_t cap = 16;
  while (cap < 2 * nnz + 16) cap <<= 1;
  hset_t h = {(int64_t *)malloc(sizeof(int64_t) * cap), cap};
  int64_t *lin = (int64_t *)malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
  if (!h.keys || !lin) { free(h.keys); free(lin); return -2; }
  memset(h.keys, 0xff, sizeof(int64_t) * cap);
  rng_t r;
  rng_init(&r, seed, 0x51ULL);
  int64_t c = 0;
  for (int64_t j = total - nnz; j < total; j++) {
    int64_t t = (int64_t)rng_below(&r, (uint64_t)(j + 1));
    if (hset_insert(&h, t)) lin[c++] = t;
    else { hset_insert(&h, j); lin[c++] = j; }
  }
  qsort(lin, (size_t)nnz, sizeof(int64_t), cmp_i64);
  for (int64_t i = 0; i <= m; i++) row_ptr[i] = 0;
  for (int64_t p = 0; p < nnz; p++) {
    row_ptr[lin[p] / n + 1]++;
    col[p] = (int32_t)(lin[p] % n);
  }
  for (int64_t i = 0; i < m; i++) row_ptr[i + 1] += row_ptr[i];
  free(h.keys);
  free(lin);
  return 0;
}

/* ---------------------------------------------------------------- power-law Omega
 * Capped power-law (Chung-Lu style) pattern:
 *   row weights  p_i ∝ rank(i)^(-a_row) over a random permutation of ranks,
 *   target degree d_i = min(n, c * p_i) with c set so that sum d_i = N
 *   (water-filling of the capped excess), rounded to integers;
 *   each row then draws d_i distinct columns with probability ∝ column weights
 *   q_j ∝ rank'(j)^(-a_col) (successive sampling without replacement).
 */
static void perm_ranks(int64_t n, uint64_t seed, uint64_t stream, double a, double *w) {
  int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * n);
  for (int64_t i = 0; i < n; i++) perm[i] = i;
  rng_t r;
  rng_init(&r, seed, stream);
  for (int64_t i = n - 1; i > 0; i--) {
    int64_t j = (int64_t)rng_below(&r, (uint64_t)(i + 1));
    int64_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
  for (int64_t i = 0; i < n; i++) w[i] = pow((double)(perm[i] + 1), -a);
  free(perm);
}

typedef struct { double f; int64_t i; } fi_t;
static int cmp_fi_desc(const void *a, const void *b) {
  const fi_t *x = (const fi_t *)a, *y = (const fi_t *)b;
  if (x->f != y->f) return (x->f < y->f) - (x->f > y->f);
  return (x->i > y->i) - (x->i < y->i);
}

/* Fills deg[m] (int64).  Returns total nnz. */
int64_t synth_powerlaw_degrees(int64_t m, int64_t n, int64_t N, double a_row, uint64_t seed,
                               int64_t *deg) {
  double *w = (double *)malloc(sizeof(double) * m);
  perm_ranks(m, seed, 0x52ULL, a_row, w);
  if (N > m * n) N = m * n;
  double lo = 0.0, hi = 1.0, wsum = 0.0;
  for (int64_t i = 0; i < m; i++) wsum += w[i];
  hi = (double)N / wsum * 4.0 + 1.0;
  for (;;) { /* grow hi until it overshoots */
    double s = 0;
    for (int64_t i = 0; i < m; i++) s += fmin((double)n, hi * w[i]);
    if (s >= (double)N) break;
    hi *= 2.0;
  }
  for (int it = 0; it < 200; it++) {
    double mid = 0.5 * (lo + hi), s = 0;
    for (int64_t i = 0; i < m; i++) s += fmin((double)n, mid * w[i]);
    if (s < (double)N) lo = mid; else hi = mid;
  }
  int64_t tot = 0;
  double *frac = (double *)malloc(sizeof(double) * m);
  for (int64_t i = 0; i < m; i++) {
    double t = fmin((double)n, hi * w[i]);
    deg[i] = (int64_t)floor(t);
    frac[i] = t - (double)deg[i];
    tot += deg[i];
  }
  /* hand out the rounding remainder to the largest fractional parts (ties by index) */
  if (tot < N) {
    fi_t *order = (fi_t *)malloc(sizeof(fi_t) * m);
    for (int64_t i = 0; i < m; i++) { order[i].f = deg[i] < n ? frac[i] : -1.0; order[i].i = i; }
    qsort(order, (size_t)m, sizeof(fi_t), cmp_fi_desc);
    for (int64_t t = 0; t < m && tot < N; t++)
      if (deg[order[t].i] < n) { deg[order[t].i]++; tot++; }
    free(order);
  }
  free(w);
  free(frac);
  return tot;
}

/* Vose alias table */
typedef struct { double *prob; int32_t *alias; int64_t n; } alias_t;
static void alias_build(alias_t *t, const double *w, int64_t n) {
  t->n = n;
  t->prob = (double *)malloc(sizeof(double) * n);
  t->alias = (int32_t *)malloc(sizeof(int32_t) * n);
  double s = 0;
  for (int64_t i = 0; i < n; i++) s += w[i];
  double *p = (double *)malloc(sizeof(double) * n);
  int64_t *small = (int64_t *)malloc(sizeof(int64_t) * n), *large = (int64_t *)malloc(sizeof(int64_t) * n);
  int64_t ns = 0, nl = 0;
  for (int64_t i = 0; i < n; i++) {
    p[i] = w[i] * (double)n / s;
    if (p[i] < 1.0) small[ns++] = i; else large[nl++] = i;
  }
  while (ns && nl) {
    int64_t l = small[--ns], g = large[nl - 1];
    t->prob[l] = p[l];
    t->alias[l] = (int32_t)g;
    p[g] = (p[g] + p[l]) - 1.0;
    if (p[g] < 1.0) { nl--; small[ns++] = g; }
  }
  while (nl) { int64_t g = large[--nl]; t->prob[g] = 1.0; t->alias[g] = (int32_t)g; }
  while (ns) { int64_t l = small[--ns]; t->prob[l] = 1.0; t->alias[l] = (int32_t)l; }
  free(p); free(small); free(large);
}
static inline int64_t alias_draw(const alias_t *t, rng_t *r) {
  int64_t i = (int64_t)rng_below(r, (uint64_t)t->n);
  return rng_u01(r) < t->prob[i] ? i : t->alias[i];
}

typedef struct { double key; int32_t j; } kj_t;
/* partial selection: afterwards a[0..d) holds the d largest keys (any order) */
static void select_top(kj_t *a, int64_t n, int64_t d, rng_t *r) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    double piv = a[lo + (int64_t)rng_below(r, (uint64_t)(hi - lo + 1))].key;
    int64_t i = lo, j = hi;
    while (i <= j) {
      while (a[i].key > piv) i++;
      while (a[j].key < piv) j--;
      if (i <= j) { kj_t t = a[i]; a[i] = a[j]; a[j] = t; i++; j--; }
    }
    if (d - 1 <= j) hi = j;
    else if (d - 1 >= i) lo = i;
    else break;
  }
}

/* row_ptr must already hold the prefix sums of the degrees. */
int synth_powerlaw_columns(int64_t m, int64_t n, double a_col, uint64_t seed, const int64_t *row_ptr,
                           int32_t *col) {
  double *w = (double *)malloc(sizeof(double) * n);
  perm_ranks(n, seed, 0x53ULL, a_col, w);
  alias_t at;
  alias_build(&at, w, n);
  int err = 0;
#pragma omp parallel
  {
    uint8_t *mark = (uint8_t *)calloc((size_t)n, 1);
    kj_t *kj = NULL;
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; i++) {
      int64_t d = row_ptr[i + 1] - row_ptr[i];
      int32_t *out = col + row_ptr[i];
      rng_t r;
      rng_init(&r, seed, 0x1000ULL + (uint64_t)i);
      if (d >= n) {
        for (int64_t j = 0; j < n; j++) out[j] = (int32_t)j;
        continue;
      }
      if (d > n / 64) { /* Efraimidis-Spirakis: keys log(u)/w_j, keep the d largest */
        if (!kj) kj = (kj_t *)malloc(sizeof(kj_t) * n);
        for (int64_t j = 0; j < n; j++) { kj[j].key = log(rng_u01(&r)) / w[j]; kj[j].j = (int32_t)j; }
        select_top(kj, n, d, &r);
        for (int64_t t = 0; t < d; t++) out[t] = kj[t].j;
      } else { /* successive sampling by rejection */
        int64_t c = 0;
        while (c < d) {
          int64_t j = alias_draw(&at, &r);
          if (!mark[j]) { mark[j] = 1; out[c++] = (int32_t)j; }
        }
        for (int64_t t = 0; t < d; t++) mark[out[t]] = 0;
      }
      qsort(out, (size_t)d, sizeof(int32_t), cmp_i32);
    }
    free(mark);
    free(kj);
  }
  free(at.prob); free(at.alias); free(w);
  return err;
}

/* ---------------------------------------------------------------- values
 * Ground truth A = U V^T with U (m x r), V (n x r) iid N(0, var_f); observed
 * values a_ij = clip(offset + (U V^T)_ij + e_ij, lo, hi), e_ij ~ N(0, var_e).
 * Set lo > hi to disable clipping.  U, V are written if the pointers are non-null.
 */
int synth_values(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col, int r, double var_f,
                 double var_e, double offset, double lo, double hi, uint64_t seed, double *val,
                 double *U_out, double *V_out) {
  double *U = (double *)malloc(sizeof(double) * m * (r > 0 ? r : 1));
  double *V = (double *)malloc(sizeof(double) * n * (r > 0 ? r : 1));
  double sf = sqrt(var_f), se = sqrt(var_e);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; i++) {
    rng_t g;
    rng_init(&g, seed, 0x100000000ULL + (uint64_t)i);
    for (int t = 0; t < r; t++) U[i * r + t] = sf * rng_normal(&g);
  }
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; j++) {
    rng_t g;
    rng_init(&g, seed, 0x200000000ULL + (uint64_t)j);
    for (int t = 0; t < r; t++) V[j * r + t] = sf * rng_normal(&g);
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < m; i++) {
    rng_t g;
    rng_init(&g, seed, 0x300000000ULL + (uint64_t)i);
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; p++) {
      const double *u = U + i * r, *v = V + (int64_t)col[p] * r;
      double x = offset;
      for (int t = 0; t < r; t++) x += u[t] * v[t];
      x += se * rng_normal(&g);
      if (lo <= hi) x = fmin(hi, fmax(lo, x));
      val[p] = x;
    }
  }
  if (U_out) memcpy(U_out, U, sizeof(double) * m * r);
  if (V_out) memcpy(V_out, V, sizeof(double) * n * r);
  free(U); free(V);
  return 0;
}

/* Ordered-key uniform reals in (0,1) (e.g. for request arrival times or per-problem draws). */
void synth_uniforms(uint64_t seed, uint64_t stream, int64_t count, double *out) {
  rng_t r;
  rng_init(&r, seed, stream);
  for (int64_t i = 0; i < count; i++) out[i] = rng_u01(&r);
}
