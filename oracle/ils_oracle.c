/* ils_oracle.c -- plain FP64 CPU oracle for the ILS splitting methods.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests and by the benchmark's CPU
 * baseline.  Slow on purpose: plain loops, no BLAS, no blocking.  OpenMP only
 * spreads independent columns across threads; every sum is taken in index
 * order by one thread, so results do not depend on the thread count.
 *
 * Each function names the passage of the paper it follows (Zhang & Li,
 * arXiv 2203.15340).  Readings of points the paper leaves open are marked
 * "Reading:".
 */
#include "ils_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define AT(i, j) A[(size_t)(j) * (size_t)lda + (size_t)(i)]

/* ------------------------------------------------------------------------ */
/* Counter-based PRNG.  Philox4x64 with 10 rounds, from Salmon, Moraes, Dror */
/* and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11).         */
/* ------------------------------------------------------------------------ */
static uint64_t mulhilo(uint64_t a, uint64_t b, uint64_t* hi) {
  unsigned __int128 prod = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(prod >> 64);
  return (uint64_t)prod;
}

void ora_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0, hi1;
    uint64_t lo0 = mulhilo(M0, c0, &hi0);
    uint64_t lo1 = mulhilo(M1, c2, &hi1);
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* SplitMix64 output mixer (Steele, Lea, Flood, OOPSLA'14). */
uint64_t ora_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Top 53 bits scaled to [0, 1). */
double ora_u01(uint64_t v) { return (double)(v >> 11) * (1.0 / 9007199254740992.0); }

/* floor(v * n / 2^64): an integer in [0, n). */
int64_t ora_uniform_index(uint64_t v, int64_t n) {
  uint64_t hi;
  (void)mulhilo(v, (uint64_t)n, &hi);
  return (int64_t)hi;
}

/* Index j drawn with probability weight_j / sum(weight) (Alg. 2, the column
 * choice by squared column norm; Remark 4.1 with alpha = 1).
 * Reading: prefix[] holds inclusive prefix sums taken in index order; the
 * draw is the smallest j with prefix[j] > u * prefix[n-1].  If rounding
 * leaves no such j, the last index of positive weight is returned. */
int64_t ora_weighted_index(const double* prefix, int64_t n, double u) {
  double thr = u * prefix[n - 1];
  int64_t lo = 0, hi = n; /* first j in [lo, hi) with prefix[j] > thr */
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (prefix[mid] > thr) hi = mid; else lo = mid + 1;
  }
  if (lo < n) return lo;
  int64_t j = n - 1;
  while (j > 0 && prefix[j] == prefix[j - 1]) --j;
  return j;
}

/* Reading of Alg. 5 step 8 (tau_t is drawn with equal probability among all
 * subsets of [n] with alpha_t members): every index s gets a key from a SplitMix64 stream seeded with a per-step
 * 64-bit value K (the s-th output of that stream), with its low b bits
 * (2^b >= n) replaced by s so that all keys differ and equal random parts
 * are ordered by index; tau_t is the set of the alpha_t indices with the
 * smallest keys.  With i.i.d. random keys every alpha_t-subset is equally
 * likely. */
static int index_bits(int64_t n) {
  int b = 1;
  while (b < 63 && ((int64_t)1 << b) < n) ++b;
  return b;
}

uint64_t ora_scd_key(uint64_t K, int64_t n, int64_t s) {
  int b = index_bits(n);
  uint64_t h = ora_mix64(K + (uint64_t)(s + 1) * 0x9E3779B97F4A7C15ull);
  return ((h >> b) << b) | (uint64_t)s;
}

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

/* member[s] = 1 for the alpha indices with the smallest keys. */
static void subset_smallest_keys(uint64_t K, int64_t n, int64_t alpha, uint8_t* member,
                                 uint64_t* scratch) {
  for (int64_t s = 0; s < n; ++s) scratch[s] = ora_scd_key(K, n, s);
  qsort(scratch, (size_t)n, sizeof(uint64_t), cmp_u64);
  memset(member, 0, (size_t)n);
  uint64_t low = (index_bits(n) >= 64) ? ~0ull : ((1ull << index_bits(n)) - 1ull);
  for (int64_t i = 0; i < alpha; ++i) member[scratch[i] & low] = 1;
}

/* PRNG addressing: one Philox block per inner step.
 * counter = (t, outer + stream_offset, 0, 0), key = (seed, method tag). */
#define TAG_RK 0x524B524753ull  /* "RKRGS" */
#define TAG_SCD 0x534344ull     /* "SCD" */

static void draw_block(uint64_t seed, uint64_t tag, uint64_t outer, uint64_t t, uint64_t out[4]) {
  uint64_t ctr[4] = {t, outer, 0, 0};
  uint64_t key[2] = {seed, tag};
  ora_philox4x64_10(ctr, key, out);
}

static void prefix_sums(const double* w, int64_t n, double* prefix) {
  double s = 0.0;
  for (int64_t j = 0; j < n; ++j) { s += w[j]; prefix[j] = s; }
}

void ora_rk_indices(uint64_t seed, uint64_t outer, int64_t t0, int64_t count,
                    const double* weights, int64_t n, int64_t* j1, int64_t* j2) {
  double* prefix = (double*)malloc(sizeof(double) * (size_t)n);
  prefix_sums(weights, n, prefix);
  for (int64_t i = 0; i < count; ++i) {
    uint64_t out[4];
    draw_block(seed, TAG_RK, outer, (uint64_t)(t0 + i), out);
    j1[i] = ora_weighted_index(prefix, n, ora_u01(out[0]));
    j2[i] = ora_weighted_index(prefix, n, ora_u01(out[1]));
  }
  free(prefix);
}

static int64_t scd_alpha(const uint64_t out[4], int64_t n, int64_t alpha_opt) {
  if (alpha_opt > 0) return alpha_opt < n ? alpha_opt : n;
  return 1 + ora_uniform_index(out[0], n);  /* alpha_t uniform on {1..n} */
}

void ora_scd_subset(uint64_t seed, uint64_t outer, int64_t t, int64_t n, int64_t alpha_opt,
                    int64_t* alpha_out, uint8_t* member) {
  uint64_t out[4];
  uint64_t* scratch = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  draw_block(seed, TAG_SCD, outer, (uint64_t)t, out);
  int64_t alpha = scd_alpha(out, n, alpha_opt);
  *alpha_out = alpha;
  subset_smallest_keys(out[2], n, alpha, member, scratch);
  free(scratch);
}

/* ------------------------------------------------------------------------ */
/* Plain dense building blocks                                              */
/* ------------------------------------------------------------------------ */

/* G = A[r0:r1, :]^T A[r0:r1, :], full symmetric n x n (Alg. 1 steps 2-3:
 * A1^T A1 and A2^T A2). */
void ora_gram(int64_t r0, int64_t r1, int64_t n, const double* A, int64_t lda, double* G) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t j = 0; j < n; ++j) {
    for (int64_t i = j; i < n; ++i) {
      double s = 0.0;
      for (int64_t k = r0; k < r1; ++k) s += AT(k, i) * AT(k, j);
      G[(size_t)j * n + i] = s;
    }
  }
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = j + 1; i < n; ++i) G[(size_t)i * n + j] = G[(size_t)j * n + i];
}

/* g = A^T J b = A1^T b1 - A2^T b2 (Alg. 1 step 4, Alg. 2 step 3). */
void ora_atjb(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda, const double* b,
              double* g) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = 0; i < p; ++i) s1 += AT(i, j) * b[i];
    for (int64_t i = p; i < p + q; ++i) s2 += AT(i, j) * b[i];
    g[j] = s1 - s2;
  }
}

/* r = A^T J (b - A x), the residual of the normal equation (Sec12). */
void ora_residual(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                  const double* b, const double* x, double* r) {
  int64_t m = p + q;
  double* t = (double*)malloc(sizeof(double) * (size_t)m);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += AT(i, j) * x[j];
    t[i] = b[i] - s;
  }
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = 0; i < p; ++i) s1 += AT(i, j) * t[i];
    for (int64_t i = p; i < m; ++i) s2 += AT(i, j) * t[i];
    r[j] = s1 - s2;
  }
  free(t);
}

static double dot(const double* a, const double* b, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

static double nrm2(const double* a, int64_t n) { return sqrt(dot(a, a, n)); }

/* RR = ||A^T J (A x - b)||^2 / ||A^T J b||^2, the stopping quantity of Sec. 5. */
double ora_rr(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
              const double* b, const double* x) {
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* g = (double*)malloc(sizeof(double) * (size_t)n);
  ora_residual(p, q, n, A, lda, b, x, r);
  ora_atjb(p, q, n, A, lda, b, g);
  double num = dot(r, r, n), den = dot(g, g, n);
  free(r);
  free(g);
  return num / den;
}

/* Cholesky G = L L^T (L lower, column-major n x n, strict upper set to 0).
 * Returns ORA_ERR_NOT_SPD on a pivot that is not > 0 (NaN included). */
int ora_cholesky(int64_t n, const double* G, double* L) {
  /* column-by-column (left-looking) Cholesky.  The rows of L are kept in a
     row-major copy R (R[i n + k] = L_ik) so that the inner products over k
     read contiguous memory; the sums are the same, in the same order. */
  double* R = (double*)calloc((size_t)n * (size_t)n, sizeof(double));
  int st = ORA_OK;
  for (int64_t j = 0; j < n && st == ORA_OK; ++j) {
    const double* Rj = R + (size_t)j * n;
    double d = G[(size_t)j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= Rj[k] * Rj[k];
    if (!(d > 0.0)) { st = ORA_ERR_NOT_SPD; break; }
    double ljj = sqrt(d);
    R[(size_t)j * n + j] = ljj;
    /* the entries below the diagonal of column j are independent of each other */
#pragma omp parallel for schedule(static) if (n - j > 256)
    for (int64_t i = j + 1; i < n; ++i) {
      const double* Ri = R + (size_t)i * n;
      double s = G[(size_t)j * n + i];
      for (int64_t k = 0; k < j; ++k) s -= Ri[k] * Rj[k];
      R[(size_t)i * n + j] = s / ljj;
    }
  }
  if (st == ORA_OK) {
    memset(L, 0, sizeof(double) * (size_t)n * (size_t)n);
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = j; i < n; ++i) L[(size_t)j * n + i] = R[(size_t)i * n + j];
  }
  free(R);
  return st;
}

/* x = (L L^T)^{-1} rhs by forward then backward substitution. */
void ora_chol_solve(int64_t n, const double* L, const double* rhs, double* x) {
  double* y = (double*)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    double s = rhs[i];
    for (int64_t k = 0; k < i; ++k) s -= L[(size_t)k * n + i] * y[k];
    y[i] = s / L[(size_t)i * n + i];
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int64_t k = i + 1; k < n; ++k) s -= L[(size_t)i * n + k] * x[k];
    x[i] = s / L[(size_t)i * n + i];
  }
  free(y);
}

/* y = G x for a column-major n x n matrix G. */
static void matvec(int64_t n, const double* G, const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += G[(size_t)j * n + i] * x[j];
    y[i] = s;
  }
}

static int all_finite(const double* v, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

static int inputs_finite(int64_t m, int64_t n, const double* A, int64_t lda, const double* b) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < m; ++i)
      if (!isfinite(AT(i, j))) return 0;
  return all_finite(b, m);
}

/* ------------------------------------------------------------------------ */
/* Direct solutions                                                         */
/* ------------------------------------------------------------------------ */

/* x_ILS = (A^T J A)^{-1} A^T J b: form the normal equation (Sec12) with plain
 * loops and solve it by Cholesky; it is SPD exactly when the ILS problem has a
 * unique solution (Sec13). */
int ora_normal_solve(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                     const double* b, double* x) {
  int64_t m = p + q;
  double* H = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
  double* L = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
  double* g = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int64_t k = 0; k < m; ++k) s += (k < p ? 1.0 : -1.0) * AT(k, i) * AT(k, j);
      H[(size_t)j * n + i] = s;
    }
  ora_atjb(p, q, n, A, lda, b, g);
  int st = ora_cholesky(n, H, L);
  if (st == ORA_OK) ora_chol_solve(n, L, g, x);
  free(H);
  free(L);
  free(g);
  return st;
}

/* QR-Cholesky method of Chandrasekaran, Gu and Sayed (1998), as summarised in
 * Sec. 1: A = QR (Householder, thin Q), solve (Q^T J Q) y = Q^T J b by
 * Cholesky, then x = R^{-1} y.  An independent route to x_ILS. */
int ora_qr_cholesky(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                    const double* b, double* x) {
  int64_t m = p + q;
  double* R = (double*)malloc(sizeof(double) * (size_t)m * (size_t)n); /* working copy */
  double* V = (double*)calloc((size_t)m * (size_t)n, sizeof(double));  /* reflectors */
  double* Q = (double*)calloc((size_t)m * (size_t)n, sizeof(double));
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < m; ++i) R[(size_t)j * m + i] = AT(i, j);
  for (int64_t k = 0; k < n; ++k) {
    double nx = 0.0;
    for (int64_t i = k; i < m; ++i) nx += R[(size_t)k * m + i] * R[(size_t)k * m + i];
    nx = sqrt(nx);
    double x0 = R[(size_t)k * m + k];
    double alpha = (x0 >= 0.0) ? -nx : nx;
    double* v = V + (size_t)k * m;
    for (int64_t i = k; i < m; ++i) v[i] = R[(size_t)k * m + i];
    v[k] -= alpha;
    double vv = 0.0;
    for (int64_t i = k; i < m; ++i) vv += v[i] * v[i];
    if (vv > 0.0) {
      for (int64_t j = k; j < n; ++j) {
        double s = 0.0;
        for (int64_t i = k; i < m; ++i) s += v[i] * R[(size_t)j * m + i];
        s = 2.0 * s / vv;
        for (int64_t i = k; i < m; ++i) R[(size_t)j * m + i] -= s * v[i];
      }
    }
    double* vk = v; /* normalise so that H = I - 2 v v^T */
    double vn = sqrt(vv);
    if (vn > 0.0)
      for (int64_t i = k; i < m; ++i) vk[i] /= vn;
  }
  /* Q = H_0 H_1 ... H_{n-1} applied to the first n columns of I_m. */
  for (int64_t j = 0; j < n; ++j) Q[(size_t)j * m + j] = 1.0;
  for (int64_t k = n - 1; k >= 0; --k) {
    const double* v = V + (size_t)k * m;
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t i = k; i < m; ++i) s += v[i] * Q[(size_t)j * m + i];
      for (int64_t i = k; i < m; ++i) Q[(size_t)j * m + i] -= 2.0 * s * v[i];
    }
  }
  double* T = (double*)calloc((size_t)n * (size_t)n, sizeof(double));
  double* L = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
  double* c = (double*)malloc(sizeof(double) * (size_t)n);
  double* y = (double*)malloc(sizeof(double) * (size_t)n);
  for (int64_t j = 0; j < n; ++j) {
    for (int64_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int64_t k = 0; k < m; ++k)
        s += (k < p ? 1.0 : -1.0) * Q[(size_t)i * m + k] * Q[(size_t)j * m + k];
      T[(size_t)j * n + i] = s;
    }
    double s = 0.0;
    for (int64_t k = 0; k < m; ++k) s += (k < p ? 1.0 : -1.0) * Q[(size_t)j * m + k] * b[k];
    c[j] = s;
  }
  int st = ora_cholesky(n, T, L);
  if (st == ORA_OK) {
    ora_chol_solve(n, L, c, y);
    for (int64_t i = n - 1; i >= 0; --i) { /* R x = y, R upper */
      double s = y[i];
      for (int64_t k = i + 1; k < n; ++k) s -= R[(size_t)k * m + i] * x[k];
      x[i] = s / R[(size_t)i * m + i];
    }
  }
  free(R); free(V); free(Q); free(T); free(L); free(c); free(y);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Shared outer-loop pieces                                                 */
/* ------------------------------------------------------------------------ */

void ora_opts_default(ora_opts* o) {
  memset(o, 0, sizeof(*o));
  o->tol = 1e-6;                  /* Sec. 5: RR < 1e-6 */
  o->stop_rule = ORA_STOP_RR;
  o->form = ORA_FORM_PAPER;
  o->variant = 0;
  o->sampling = ORA_SAMPLE_UNIFORM;
  o->max_outer = 20000;           /* Sec. 5: at most 20000 outer iterations */
  o->max_inner = -1;              /* -1: 1000 * n */
  o->inner_tol = -1.0;            /* -1: 1e-8 paper form, 1e-2 correction form */
  o->inner_check = -1;            /* -1: n */
  o->seed = 0;
  o->stream_offset = 0;
  o->alpha = 0;
}

static int check_args(int64_t p, int64_t q, int64_t n, int64_t lda, const double* A,
                      const double* b, const double* x, const ora_opts* o) {
  if (!A || !b || !x || !o) return ORA_ERR_ARG;
  if (n < 1 || q < 0 || p < n || lda < p + q) return ORA_ERR_ARG;
  if (o->stop_rule < 0 || o->stop_rule > 2) return ORA_ERR_ARG;
  if (o->stop_rule != ORA_STOP_FIXED && !(o->tol > 0.0)) return ORA_ERR_ARG;
  if (o->stop_rule == ORA_STOP_XREF && !o->x_ref) return ORA_ERR_ARG;
  if (o->max_outer < 0) return ORA_ERR_ARG;
  if (o->form != ORA_FORM_PAPER && o->form != ORA_FORM_CORRECTION) return ORA_ERR_ARG;
  return ORA_OK;
}

/* Outer stopping quantity at x_k: RR (Sec. 5) or the relative error. */
static double outer_metric(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                           const double* b, const double* x, const ora_opts* o) {
  if (o->stop_rule == ORA_STOP_XREF) {
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double d = x[i] - o->x_ref[i];
      num += d * d;
      den += o->x_ref[i] * o->x_ref[i];
    }
    return sqrt(num) / sqrt(den);
  }
  return ora_rr(p, q, n, A, lda, b, x);
}

static void finish_info(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                        const double* b, const double* x, const ora_opts* o, int st,
                        int64_t outer, int64_t inner, ora_info* info) {
  if (!info) return;
  info->status = st;
  info->outer_iters = outer;
  info->inner_iters = inner;
  info->rr = ora_rr(p, q, n, A, lda, b, x);
  info->rel_err = -1.0;
  if (o->x_ref) {
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double d = x[i] - o->x_ref[i];
      num += d * d;
      den += o->x_ref[i] * o->x_ref[i];
    }
    info->rel_err = sqrt(num) / sqrt(den);
  }
}

static double default_inner_tol(const ora_opts* o) {
  if (o->inner_tol > 0.0) return o->inner_tol;
  return o->form == ORA_FORM_CORRECTION ? 1e-2 : 1e-8;
}

/* ------------------------------------------------------------------------ */
/* SP, Algorithm 1 and update (Sec23)                                       */
/* ------------------------------------------------------------------------ */

/* x_{k+1} = (A1^T A1)^{-1} A2^T A2 x_k + (A1^T A1)^{-1} A^T J b  (Sec23).
 * ORA_SP_EXPLICIT forms the iteration matrix and constant of (Sec23) once,
 * B = (A1^T A1)^{-1} A2^T A2 and c = (A1^T A1)^{-1} A^T J b (the inverse by
 * Cholesky solves against the unit vectors), then x <- B x + c.
 * ORA_SP_CHOLESKY applies (A1^T A1)^{-1} by two triangular solves per step.  The correction form solves
 * A1^T A1 d = A^T J (b - A x_k) and sets x_{k+1} = x_k + d, the same iterate
 * in exact arithmetic (subtract A1^T A1 x_k from both sides of (Sec23) and use
 * A^T J A = A1^T A1 - A2^T A2). */
int ora_sp_solve(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                 const double* b, const double* x0, double* x, const ora_opts* o,
                 ora_info* info) {
  int st = check_args(p, q, n, lda, A, b, x, o);
  if (st != ORA_OK) { if (info) info->status = st; return st; }
  int64_t m = p + q;
  if (!inputs_finite(m, n, A, lda, b)) { if (info) info->status = ORA_ERR_NONFINITE; return ORA_ERR_NONFINITE; }
  size_t nn = (size_t)n * (size_t)n;
  double* G1 = (double*)malloc(sizeof(double) * nn);
  double* G2 = (double*)malloc(sizeof(double) * nn);
  double* L = (double*)malloc(sizeof(double) * nn);
  double* P = NULL;
  double* B = NULL;
  double* g = (double*)malloc(sizeof(double) * (size_t)n);
  double* c = (double*)malloc(sizeof(double) * (size_t)n);
  double* xk = (double*)malloc(sizeof(double) * (size_t)n);
  double* t1 = (double*)malloc(sizeof(double) * (size_t)n);
  double* t2 = (double*)malloc(sizeof(double) * (size_t)n);
  ora_gram(0, p, n, A, lda, G1);
  ora_gram(p, m, n, A, lda, G2);
  ora_atjb(p, q, n, A, lda, b, g);
  st = ora_cholesky(n, G1, L);
  int64_t k = 0;
  if (st != ORA_OK) goto done;
  if (o->variant == ORA_SP_EXPLICIT) {
    P = (double*)malloc(sizeof(double) * nn);
    B = (double*)malloc(sizeof(double) * nn);
    double* e = t1;
    for (int64_t j = 0; j < n; ++j) { /* P = G1^{-1}, column by column */
      for (int64_t i = 0; i < n; ++i) e[i] = (i == j) ? 1.0 : 0.0;
      ora_chol_solve(n, L, e, P + (size_t)j * n);
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) /* B = P G2 */
      for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t l = 0; l < n; ++l) s += P[(size_t)l * n + i] * G2[(size_t)j * n + l];
        B[(size_t)j * n + i] = s;
      }
    matvec(n, P, g, c); /* c = P g */
  }
  for (int64_t i = 0; i < n; ++i) xk[i] = x0 ? x0[i] : 0.0;
  st = ORA_OK;
  for (k = 0;; ++k) {
    if (o->stop_rule != ORA_STOP_FIXED && outer_metric(p, q, n, A, lda, b, xk, o) < o->tol) break;
    if (k == o->max_outer) {
      if (o->stop_rule != ORA_STOP_FIXED) st = ORA_ERR_NO_CONVERGENCE;
      break;
    }
    if (o->form == ORA_FORM_PAPER) {
      if (o->variant == ORA_SP_EXPLICIT) {
        matvec(n, B, xk, t1);
        for (int64_t i = 0; i < n; ++i) xk[i] = t1[i] + c[i];
      } else {
        matvec(n, G2, xk, t1);
        for (int64_t i = 0; i < n; ++i) t1[i] += g[i];
        ora_chol_solve(n, L, t1, xk);
      }
    } else {
      ora_residual(p, q, n, A, lda, b, xk, t1);
      if (o->variant == ORA_SP_EXPLICIT) matvec(n, P, t1, t2);
      else ora_chol_solve(n, L, t1, t2);
      for (int64_t i = 0; i < n; ++i) xk[i] += t2[i];
    }
    if (!all_finite(xk, n)) { st = ORA_ERR_NONFINITE; ++k; break; }
  }
  memcpy(x, xk, sizeof(double) * (size_t)n);
done:
  if (st == ORA_ERR_NOT_SPD) { if (info) info->status = st; }
  else finish_info(p, q, n, A, lda, b, x, o, st, k, 0, info);
  free(G1); free(G2); free(L); free(P); free(B); free(g); free(c); free(xk); free(t1); free(t2);
  return st;
}

/* ------------------------------------------------------------------------ */
/* SP-RK-RGS, Algorithm 2                                                   */
/* ------------------------------------------------------------------------ */

/* The two one-dimensional projections the method is built from.
 * Kaczmarz half (eq. Sec3.32111, A1^T w = bhat): move w to the nearest point
 * of the hyperplane {y : a^T y = beta}, a = A1_(j1), beta = bhat_j1; that is
 * w + gamma a with gamma = (beta - a^T w) / ||a||^2.  Returns gamma. */
static double kaczmarz_project(double* w, const double* a, double beta, double a_nrm2, int64_t p) {
  double gamma = (beta - dot(a, w, p)) / a_nrm2;
  for (int64_t i = 0; i < p; ++i) w[i] += gamma * a[i];
  return gamma;
}

/* Gauss-Seidel half (eq. Sec3.33111, A1 z = w): z_j2 changes by the delta
 * that minimises ||v - delta a||, v = w - A1 z the current misfit and
 * a = A1_(j2): delta = a^T v / ||a||^2. */
static double gs_line_min(const double* a, const double* v, double a_nrm2, int64_t p) {
  return dot(a, v, p) / a_nrm2;
}

/* SP-RK-RGS.  Outer right-hand side bhat = A2^T A2 x_k + A^T J b (the SP
 * update (Sec23) with A1^T A1 left to the inner solver), or in the correction
 * form the residual A^T J (b - A x_k).  The inner solver approaches the
 * solution of A1^T A1 z = bhat, the fixed point of Thm 3.1, from w = z = 0 by
 * alternating the two projections above, each on a column drawn with
 * probability ||A1_(j)||^2 / ||A1||_F^2 (j1 first, then j2, independently).
 * LITERAL forms the misfit w - A1 z afresh for every Gauss-Seidel half (the
 * work counted in the cost remark after Alg. 2).  INCREMENTAL carries
 * s = w - A1 z instead: s gains the Kaczmarz move gamma a1 and loses the
 * Gauss-Seidel move delta a2; the iterates are the same in exact arithmetic.
 * Reading (the inner loops run to convergence): every inner_check steps, starting at
 * t = 0, stop if ||bhat - A1^T A1 z|| <= inner_tol * ||bhat|| (INCREMENTAL uses
 * A1 z = w - s); always stop after max_inner steps.  ORA_STOP_FIXED runs
 * exactly max_inner inner steps and max_outer outer steps. */
int ora_rk_solve(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                 const double* b, const double* x0, double* x, const ora_opts* o,
                 ora_info* info) {
  int st = check_args(p, q, n, lda, A, b, x, o);
  if (st != ORA_OK) { if (info) info->status = st; return st; }
  int64_t m = p + q;
  if (!inputs_finite(m, n, A, lda, b)) { if (info) info->status = ORA_ERR_NONFINITE; return ORA_ERR_NONFINITE; }
  int64_t max_inner = o->max_inner >= 0 ? o->max_inner : 1000 * n;
  int64_t check = o->inner_check > 0 ? o->inner_check : n;
  double itol = default_inner_tol(o);
  size_t nn = (size_t)n * (size_t)n;
  double* G2 = (double*)malloc(sizeof(double) * nn);
  double* g = (double*)malloc(sizeof(double) * (size_t)n);
  double* cn = (double*)malloc(sizeof(double) * (size_t)n);
  double* prefix = (double*)malloc(sizeof(double) * (size_t)n);
  double* xk = (double*)malloc(sizeof(double) * (size_t)n);
  double* tgt = (double*)malloc(sizeof(double) * (size_t)n);
  double* z = (double*)malloc(sizeof(double) * (size_t)n);
  double* res = (double*)malloc(sizeof(double) * (size_t)n);
  double* w = (double*)malloc(sizeof(double) * (size_t)p);
  double* s = (double*)malloc(sizeof(double) * (size_t)p);
  double* v = (double*)malloc(sizeof(double) * (size_t)p);
  ora_gram(p, m, n, A, lda, G2);
  ora_atjb(p, q, n, A, lda, b, g);
  for (int64_t j = 0; j < n; ++j) {
    double t = 0.0;
    for (int64_t i = 0; i < p; ++i) t += AT(i, j) * AT(i, j);
    cn[j] = t;
  }
  int64_t k = 0, inner_total = 0;
  for (int64_t j = 0; j < n; ++j)
    if (!(cn[j] > 0.0)) { st = ORA_ERR_NOT_SPD; goto done; }  /* zero column: A1 rank deficient */
  prefix_sums(cn, n, prefix);
  for (int64_t i = 0; i < n; ++i) xk[i] = x0 ? x0[i] : 0.0;
  st = ORA_OK;
  for (k = 0;; ++k) {
    if (o->stop_rule != ORA_STOP_FIXED && outer_metric(p, q, n, A, lda, b, xk, o) < o->tol) break;
    if (k == o->max_outer) {
      if (o->stop_rule != ORA_STOP_FIXED) st = ORA_ERR_NO_CONVERGENCE;
      break;
    }
    if (o->form == ORA_FORM_PAPER) {
      matvec(n, G2, xk, tgt);
      for (int64_t i = 0; i < n; ++i) tgt[i] += g[i];
    } else {
      ora_residual(p, q, n, A, lda, b, xk, tgt);
    }
    double tn = nrm2(tgt, n);
    memset(w, 0, sizeof(double) * (size_t)p);
    memset(s, 0, sizeof(double) * (size_t)p);
    memset(z, 0, sizeof(double) * (size_t)n);
    int64_t t = 0;
    for (;;) {
      if (o->stop_rule != ORA_STOP_FIXED && t % check == 0) {
        /* res = bhat - A1^T (A1 z) */
        if (o->variant == ORA_RK_LITERAL) {
          for (int64_t i = 0; i < p; ++i) {
            double acc = 0.0;
            for (int64_t j = 0; j < n; ++j) acc += AT(i, j) * z[j];
            v[i] = acc;
          }
        } else {
          for (int64_t i = 0; i < p; ++i) v[i] = w[i] - s[i];
        }
        for (int64_t j = 0; j < n; ++j) {
          double acc = 0.0;
          for (int64_t i = 0; i < p; ++i) acc += AT(i, j) * v[i];
          res[j] = tgt[j] - acc;
        }
        if (nrm2(res, n) <= itol * tn) break;
      }
      if (t == max_inner) break;
      uint64_t out[4];
      draw_block(o->seed, TAG_RK, (uint64_t)k + o->stream_offset, (uint64_t)t, out);
      int64_t j1 = ora_weighted_index(prefix, n, ora_u01(out[0]));
      int64_t j2 = ora_weighted_index(prefix, n, ora_u01(out[1]));
      const double* a1 = A + (size_t)j1 * (size_t)lda;
      const double* a2 = A + (size_t)j2 * (size_t)lda;
      const double gamma = kaczmarz_project(w, a1, tgt[j1], cn[j1], p);
      double delta;
      if (o->variant == ORA_RK_LITERAL) {
        for (int64_t i = 0; i < p; ++i) { /* v = w - A1 z */
          double acc = 0.0;
          for (int64_t j = 0; j < n; ++j) acc += AT(i, j) * z[j];
          v[i] = w[i] - acc;
        }
        delta = gs_line_min(a2, v, cn[j2], p);
        z[j2] += delta;
      } else {
        for (int64_t i = 0; i < p; ++i) s[i] += gamma * a1[i];
        delta = gs_line_min(a2, s, cn[j2], p);
        z[j2] += delta;
        for (int64_t i = 0; i < p; ++i) s[i] -= delta * a2[i];
      }
      ++t;
    }
    inner_total += t;
    if (o->form == ORA_FORM_PAPER) memcpy(xk, z, sizeof(double) * (size_t)n);
    else for (int64_t i = 0; i < n; ++i) xk[i] += z[i];
    if (!all_finite(xk, n)) { st = ORA_ERR_NONFINITE; ++k; break; }
  }
  memcpy(x, xk, sizeof(double) * (size_t)n);
done:
  if (st == ORA_ERR_NOT_SPD) { if (info) info->status = st; }
  else finish_info(p, q, n, A, lda, b, x, o, st, k, inner_total, info);
  free(G2); free(g); free(cn); free(prefix); free(xk); free(tgt); free(z); free(res);
  free(w); free(s); free(v);
  return st;
}

/* ------------------------------------------------------------------------ */
/* SP-SCD, Algorithm 5 (the practical form run in Sec. 5)                   */
/* ------------------------------------------------------------------------ */

/* Outer as in Algorithm 2.  Inner from beta = 0, r = bhat:
 *   alpha_t at random in [n]; tau_t a uniform alpha_t-subset of [n];
 *   j = argmax_{s in tau_t} |r_s|; r -= r_j / G1_jj * G1_(j); beta_j += r_j / G1_jj.
 * Readings: alpha_t is uniform on {1..n} (or fixed by opts.alpha); tau_t holds
 * the alpha_t indices with the smallest keys ora_scd_key(K_t, n, .); the
 * argmax takes the smallest index among equal |r_s|; the update uses the
 * current r_t (the printed r_k^{(j_t)} indexes the inner step).  With
 * ORA_SAMPLE_NORM and alpha = 1, j is drawn with probability
 * G1_jj / trace(G1) instead (the SP-RCD case of Remark 4.1).
 * Inner stop: before every step, stop if ||r|| <= inner_tol * ||bhat||;
 * always stop after max_inner steps. */
int ora_rgs_solve(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                  const double* b, const double* x0, double* x, const ora_opts* o,
                  ora_info* info) {
  int st = check_args(p, q, n, lda, A, b, x, o);
  if (st != ORA_OK) { if (info) info->status = st; return st; }
  if (o->sampling == ORA_SAMPLE_NORM && o->alpha != 1) { if (info) info->status = ORA_ERR_ARG; return ORA_ERR_ARG; }
  int64_t m = p + q;
  if (!inputs_finite(m, n, A, lda, b)) { if (info) info->status = ORA_ERR_NONFINITE; return ORA_ERR_NONFINITE; }
  int64_t max_inner = o->max_inner >= 0 ? o->max_inner : 1000 * n;
  double itol = default_inner_tol(o);
  size_t nn = (size_t)n * (size_t)n;
  double* G1 = (double*)malloc(sizeof(double) * nn);
  double* G2 = (double*)malloc(sizeof(double) * nn);
  double* L = (double*)malloc(sizeof(double) * nn);
  double* g = (double*)malloc(sizeof(double) * (size_t)n);
  double* diag = (double*)malloc(sizeof(double) * (size_t)n);
  double* prefix = (double*)malloc(sizeof(double) * (size_t)n);
  double* xk = (double*)malloc(sizeof(double) * (size_t)n);
  double* tgt = (double*)malloc(sizeof(double) * (size_t)n);
  double* beta = (double*)malloc(sizeof(double) * (size_t)n);
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  uint8_t* member = (uint8_t*)malloc((size_t)n);
  ora_gram(0, p, n, A, lda, G1);
  ora_gram(p, m, n, A, lda, G2);
  ora_atjb(p, q, n, A, lda, b, g);
  int64_t k = 0, inner_total = 0;
  st = ora_cholesky(n, G1, L); /* only to report a matrix that is not SPD */
  if (st != ORA_OK) goto done;
  for (int64_t j = 0; j < n; ++j) diag[j] = G1[(size_t)j * n + j];
  prefix_sums(diag, n, prefix);
  for (int64_t i = 0; i < n; ++i) xk[i] = x0 ? x0[i] : 0.0;
  for (k = 0;; ++k) {
    if (o->stop_rule != ORA_STOP_FIXED && outer_metric(p, q, n, A, lda, b, xk, o) < o->tol) break;
    if (k == o->max_outer) {
      if (o->stop_rule != ORA_STOP_FIXED) st = ORA_ERR_NO_CONVERGENCE;
      break;
    }
    if (o->form == ORA_FORM_PAPER) {
      matvec(n, G2, xk, tgt);
      for (int64_t i = 0; i < n; ++i) tgt[i] += g[i];
    } else {
      ora_residual(p, q, n, A, lda, b, xk, tgt);
    }
    double tn = nrm2(tgt, n);
    memset(beta, 0, sizeof(double) * (size_t)n);
    memcpy(r, tgt, sizeof(double) * (size_t)n);
    int64_t t = 0;
    for (;;) {
      if (o->stop_rule != ORA_STOP_FIXED && nrm2(r, n) <= itol * tn) break;
      if (t == max_inner) break;
      uint64_t out[4];
      draw_block(o->seed, TAG_SCD, (uint64_t)k + o->stream_offset, (uint64_t)t, out);
      int64_t j = -1;
      if (o->sampling == ORA_SAMPLE_NORM) {
        j = ora_weighted_index(prefix, n, ora_u01(out[1]));
      } else {
        int64_t alpha = scd_alpha(out, n, o->alpha);
        subset_smallest_keys(out[2], n, alpha, member, keys);
        double best = -1.0;
        for (int64_t s2 = 0; s2 < n; ++s2) {
          if (!member[s2]) continue;
          double a = fabs(r[s2]);
          if (a > best) { best = a; j = s2; }
        }
      }
      if (j < 0) break; /* only reachable when r is not finite */
      double gamma = r[j] / G1[(size_t)j * n + j];
      const double* col = G1 + (size_t)j * n;
      for (int64_t i = 0; i < n; ++i) r[i] -= gamma * col[i];
      beta[j] += gamma;
      ++t;
    }
    inner_total += t;
    if (o->form == ORA_FORM_PAPER) memcpy(xk, beta, sizeof(double) * (size_t)n);
    else for (int64_t i = 0; i < n; ++i) xk[i] += beta[i];
    if (!all_finite(xk, n)) { st = ORA_ERR_NONFINITE; ++k; break; }
  }
  memcpy(x, xk, sizeof(double) * (size_t)n);
done:
  if (st == ORA_ERR_NOT_SPD) { if (info) info->status = st; }
  else finish_info(p, q, n, A, lda, b, x, o, st, k, inner_total, info);
  free(G1); free(G2); free(L); free(g); free(diag); free(prefix); free(xk); free(tgt);
  free(beta); free(r); free(keys); free(member);
  return st;
}

/* Worker threads of the OpenMP loops (timing runs of the oracle only; the
 * results do not depend on the count: every parallel loop writes disjoint
 * entries and each entry's sum runs in index order). */
void ora_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
int ora_max_threads(void) { return omp_get_max_threads(); }
