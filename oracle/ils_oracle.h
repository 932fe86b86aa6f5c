/* ils_oracle.h -- plain FP64 CPU oracle for the indefinite least squares
 * (ILS) splitting methods of Zhang & Li, "Splitting-based randomized iterative
 * methods for solving indefinite least squares problem" (arXiv 2203.15340).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests and the
 * benchmark's CPU-baseline leg can check and time the GPU solver against a
 * slow, obviously correct reference.  No product code links it.  It shares
 * no source, header or constant table with the GPU library.
 *
 * Problem (Sec. 1, eq. Sec11): min_x (b - A x)^T J (b - A x), A m x n, m >= n,
 * J = diag(I_p, -I_q), p + q = m.  A1 = rows [0,p), A2 = rows [p,m).
 * All matrices are column-major FP64 host arrays; A has leading dimension lda.
 */
#ifndef ILS_ORACLE_H
#define ILS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_OK = 0, ORA_ERR_ARG = -1, ORA_ERR_NOT_SPD = -2, ORA_ERR_NO_CONVERGENCE = -3,
       ORA_ERR_NONFINITE = -4 };
enum { ORA_STOP_RR = 0, ORA_STOP_XREF = 1, ORA_STOP_FIXED = 2 };
enum { ORA_FORM_PAPER = 0, ORA_FORM_CORRECTION = 1 };
/* SP: how G1^{-1} is applied.  EXPLICIT = the iteration matrix and constant
 * of the update (Sec23) formed once (B = G1^{-1} G2, c = G1^{-1} A^T J b).
 * CHOLESKY = two triangular solves per iteration.
 * RK-RGS: INCREMENTAL carries s = w - A1 z; LITERAL recomputes A1 z. */
enum { ORA_SP_EXPLICIT = 0, ORA_SP_CHOLESKY = 1 };
enum { ORA_RK_INCREMENTAL = 0, ORA_RK_LITERAL = 1 };
enum { ORA_SAMPLE_UNIFORM = 0, ORA_SAMPLE_NORM = 1 };

typedef struct {
  double tol;             /* outer stop threshold (RR or relative error) */
  int32_t stop_rule;      /* ORA_STOP_* */
  int32_t form;           /* ORA_FORM_* */
  int32_t variant;        /* ORA_SP_* for SP, ORA_RK_* for RK-RGS */
  int32_t sampling;       /* SCD only: ORA_SAMPLE_* */
  const double* x_ref;    /* n, required for ORA_STOP_XREF */
  int64_t max_outer;
  int64_t max_inner;
  double inner_tol;
  int64_t inner_check;    /* RK-RGS: steps between inner residual checks */
  uint64_t seed;
  uint64_t stream_offset; /* added to the outer index in the PRNG counter */
  int64_t alpha;          /* SCD: 0 = alpha_t uniform on {1..n}; k > 0 = fixed */
} ora_opts;

typedef struct {
  int32_t status;
  int32_t pad;
  int64_t outer_iters;
  int64_t inner_iters;
  double rr;              /* RR at the returned x (Sec. 5) */
  double rel_err;         /* ||x - x_ref|| / ||x_ref|| if x_ref given, else -1 */
} ora_info;

/* ---- counter-based PRNG (Philox4x64-10) and the derived draws ---- */
void ora_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
uint64_t ora_mix64(uint64_t z);
double ora_u01(uint64_t v);
int64_t ora_uniform_index(uint64_t v, int64_t n);
int64_t ora_weighted_index(const double* prefix, int64_t n, double u);
uint64_t ora_scd_key(uint64_t K, int64_t n, int64_t s);
/* index streams of the randomized inner loops, for sampler parity checks */
void ora_rk_indices(uint64_t seed, uint64_t outer, int64_t t0, int64_t count,
                    const double* weights, int64_t n, int64_t* j1, int64_t* j2);
void ora_scd_subset(uint64_t seed, uint64_t outer, int64_t t, int64_t n, int64_t alpha_opt,
                    int64_t* alpha_out, uint8_t* member);

/* ---- plain dense building blocks ---- */
void ora_gram(int64_t r0, int64_t r1, int64_t n, const double* A, int64_t lda, double* G);
void ora_atjb(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda, const double* b,
              double* g);
void ora_residual(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                  const double* b, const double* x, double* r);
double ora_rr(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
              const double* b, const double* x);
int ora_cholesky(int64_t n, const double* G, double* L);
void ora_chol_solve(int64_t n, const double* L, const double* rhs, double* x);

/* ---- direct solutions of the normal equation (Sec12) ---- */
int ora_normal_solve(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                     const double* b, double* x);
int ora_qr_cholesky(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                    const double* b, double* x);

/* ---- the three iterative methods ---- */
void ora_opts_default(ora_opts* o);
int ora_sp_solve(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                 const double* b, const double* x0, double* x, const ora_opts* o,
                 ora_info* info);
int ora_rk_solve(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                 const double* b, const double* x0, double* x, const ora_opts* o,
                 ora_info* info);
int ora_rgs_solve(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                  const double* b, const double* x0, double* x, const ora_opts* o,
                  ora_info* info);

/* ---- warm-start network (mlp_oracle.c): d = {d0, d1, d2, d3} ---- */
int64_t ora_mlp_nparams(const int64_t d[4]);
void ora_mlp_forward(const int64_t d[4], const double* theta, int64_t B, const double* U,
                     double* Y, double* H1, double* H2);
double ora_mlp_loss(const int64_t d[4], const double* theta, int64_t B, const double* U,
                    const double* T);
double ora_mlp_grad(const int64_t d[4], const double* theta, int64_t B, const double* U,
                    const double* T, double* grad);
void ora_adam_step(int64_t len, double* w, double* m, double* v, const double* g, int64_t t,
                   double lr, double beta1, double beta2, double eps);
double ora_bf16_round(double x);

/* ---- sparse matrices (sparse_oracle.c) ---- */
void ora_csr_to_csc(int64_t m, int64_t n, int64_t p, const int64_t* rowptr, const int32_t* colidx,
                    const double* val, int64_t* colptr, int32_t* rowidx, double* cval, int32_t* a1len);

/* OpenMP worker threads for later calls (timing only; results are the same
 * for any count). */
void ora_set_threads(int t);
int ora_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
