/* ils.h -- C ABI of the MI355X (gfx950) solver for the indefinite least
 * squares (ILS) problem by the splitting methods of Zhang & Li,
 * "Splitting-based randomized iterative methods for solving indefinite least
 * squares problem" (arXiv 2203.15340).
 *
 * Problem (Sec. 1, eq. Sec11):  min_x (b - A x)^T J (b - A x),
 *   A is m x n with m >= n, J = diag(I_p, -I_q), p + q = m.
 * Partition (eq. Sec121): A1 = rows [0, p) of A, A2 = rows [p, m); b1, b2 alike.
 * The problem has a unique solution iff A^T J A = A1^T A1 - A2^T A2 is
 * symmetric positive definite (eq. Sec13), which needs p >= n.
 *
 * Memory and layout.  Every array argument is a DEVICE pointer on the device
 * of the handle (hipMalloc'd memory or a torch tensor's data_ptr()), except
 * where marked "host".  A is column-major FP64 with leading dimension
 * lda >= m; A1 and A2 are row ranges of that one buffer.  b has m entries,
 * x0, x and x_ref have n.  The caller owns every array it passes; the
 * library neither frees nor keeps any caller pointer after a call returns.
 * The handle owns all workspace (Gram matrices, factors, vectors, sampler
 * tables), grows it on demand and frees it in ils_destroy.
 *
 * Streams and blocking.  Work is queued on the handle's stream (the one given
 * to ils_create, else a stream the handle creates).  The solve calls return
 * after that work has finished, since the iteration counts and status are
 * read back into the host ils_info.  A handle must not be used by two host
 * threads at once.
 *
 * Errors.  Calls return ILS_OK (0) or a negative ils_status; info->status
 * holds the same value.  On ILS_ERR_ARG, ILS_ERR_NONFINITE (non-finite entry
 * in A or b) and ILS_ERR_NOT_SPD x is left untouched.  On
 * ILS_ERR_NO_CONVERGENCE x holds the last iterate, which may be passed back
 * as x0 to resume: each method converges from any start (Thm 2.1, 3.2, 4.1).
 * ILS_ERR_NONFINITE is also returned when an iterate becomes non-finite; x
 * then holds that iterate.  ILS_ERR_HIP reports a failed HIP call, and also a
 * device-side wait of the one-launch elimination (n <= 2048) that ran out of
 * its bounded spin, which does not happen in normal operation; x is then left
 * untouched.
 */
#ifndef ILS_H
#define ILS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ILS_OK = 0,
  ILS_ERR_ARG = -1,            /* invalid sizes, pointers or options */
  ILS_ERR_NOT_SPD = -2,        /* A1^T A1 not positive definite (rank(A1) < n) */
  ILS_ERR_NO_CONVERGENCE = -3, /* max_outer reached before the stop rule held */
  ILS_ERR_NONFINITE = -4,      /* NaN/Inf in A, b or an iterate */
  ILS_ERR_HIP = -5,            /* a HIP runtime call failed */
  ILS_ERR_ALLOC = -6           /* device memory allocation failed */
} ils_status;

/* Outer stopping rule, checked at x_k before x_{k+1} is formed. */
enum {
  ILS_STOP_RR = 0,    /* RR = ||A^T J (A x - b)||^2 / ||A^T J b||^2 < tol (Sec. 5) */
  ILS_STOP_XREF = 1,  /* ||x - x_ref|| / ||x_ref|| < tol */
  ILS_STOP_FIXED = 2  /* exactly max_outer outer steps (and max_inner inner steps) */
};

/* Which right-hand side each outer step solves with A1^T A1. */
enum {
  ILS_FORM_PAPER = 0,      /* A1^T A1 x_{k+1} = A2^T A2 x_k + A^T J b (eq. Sec23, Sec3.41) */
  ILS_FORM_CORRECTION = 1  /* A1^T A1 d = A^T J (b - A x_k), x_{k+1} = x_k + d:
                              the same iterate in exact arithmetic, since
                              A^T J A = A1^T A1 - A2^T A2 (Sec. 2) */
};

enum {
  ILS_PREC_FP64 = 0,  /* every step in FP64 */
  ILS_PREC_MIXED = 1  /* A1^T A1 and the inner sweeps in FP32, residual and
                         update in FP64; needs ILS_FORM_CORRECTION.  SP: FP32
                         Gram of A1, FP64 elimination.  SP-RK-RGS: FP32 copy
                         of A1, FP32 w and s.  SP-SCD: FP32 A1^T A1 and FP32
                         residual r in the coordinate steps (beta FP64).
                         Dense A only. */
};

/* SP-SCD column choice (Alg. 5 and Remark 4.1). */
enum {
  ILS_SAMPLE_UNIFORM = 0, /* uniform alpha_t-subset, largest |residual| in it */
  ILS_SAMPLE_NORM = 1     /* alpha = 1 with P(j) = ||A1_(j)||^2 / ||A1||_F^2 (SP-RCD) */
};

typedef struct {
  double tol;            /* outer threshold; default 1e-6 (Sec. 5) */
  int32_t stop_rule;     /* ILS_STOP_*; default ILS_STOP_RR */
  int32_t form;          /* ILS_FORM_*; default ILS_FORM_PAPER */
  int32_t precision;     /* ILS_PREC_*; default ILS_PREC_FP64 */
  int32_t sampling;      /* ILS_SAMPLE_*; SP-SCD only */
  const double* x_ref;   /* device, n; required iff stop_rule == ILS_STOP_XREF */
  int64_t max_outer;     /* default 20000 (Sec. 5) */
  int64_t max_inner;     /* randomized methods; -1 = 1000 * n */
  double inner_tol;      /* randomized methods: stop the inner loop when
                            ||bhat - A1^T A1 z|| <= inner_tol * ||bhat||;
                            -1 = 1e-8 (paper form) or 1e-2 (correction form) */
  int64_t inner_check;   /* SP-RK-RGS: inner steps between residual checks; -1 = n */
  uint64_t seed;         /* randomized methods: Philox key */
  uint64_t stream_offset;/* added to the outer index in the Philox counter */
  int64_t alpha;         /* SP-SCD: 0 = alpha_t uniform on {1..n} (Alg. 5 step 7);
                            k > 0 = fixed alpha = min(k, n); k = n is the greedy
                            (Motzkin) choice; 1 with ILS_SAMPLE_NORM is SP-RCD */
} ils_opts;

typedef struct {
  int32_t status;        /* same as the return value */
  int32_t pad;
  int64_t outer_iters;   /* outer updates performed */
  int64_t inner_iters;   /* randomized methods: inner steps over all outer steps */
  double rr;             /* RR at the returned x when stop_rule == ILS_STOP_RR, else NaN */
  double rel_err;        /* ||x - x_ref|| / ||x_ref|| when x_ref is given, else -1 */
  double device_ms;      /* device time from the first to the last queued kernel:
                          * measured while phase timing is on
                          * (ils_set_profiling), else 0; the batched solver
                          * always measures it */
} ils_info;

typedef struct ils_handle ils_handle;

/* Create a handle bound to device_ordinal.  hip_stream is a hipStream_t (or
 * NULL, in which case the handle creates its own default-priority stream). */
int ils_create(ils_handle** h, int device_ordinal, void* hip_stream);
int ils_destroy(ils_handle* h);
/* Fill *o with the defaults listed in ils_opts. */
void ils_opts_default(ils_opts* o);
/* Static string describing a status code. */
const char* ils_status_string(int status);

/* SP method, Algorithm 1: P = (A1^T A1)^{-1}, B = P A2^T A2, c = P A^T J b,
 * x_{k+1} = B x_k + c (eq. Sec23).  B and c are formed by block Gauss-Jordan
 * elimination of [A1^T A1 | A2^T A2 | A^T J b] (P itself is never stored);
 * the correction form and the mixed precision form keep P = (A1^T A1)^{-1}
 * and iterate x_{k+1} = x_k + P A^T J (b - A x_k).
 * x0 may be NULL (zero start, as in Sec. 5) and may alias x. */
int ils_sp_solve(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                 const double* b, const double* x0, double* x, const ils_opts* opts,
                 ils_info* info /* host */);

/* SP-RK-RGS, Algorithm 2: each outer step runs randomized Kaczmarz steps on
 * A1^T w = bhat (eq. Sec3.32111) interleaved with randomized Gauss-Seidel
 * steps on A1 z = w (eq. Sec3.33111), both choosing columns of A1 with
 * probability ||A1_(j)||^2 / ||A1||_F^2, and sets x_{k+1} = z.
 * ILS_PREC_MIXED (with ILS_FORM_CORRECTION): the inner sweeps read an FP32
 * copy of A1 and keep w, s in FP32 with FP32 sums; the outer residual
 * A^T J (b - A x_k), z and x stay FP64 (iterative refinement). */
int ils_rk_solve(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                 const double* b, const double* x0, double* x, const ils_opts* opts,
                 ils_info* info /* host */);

/* SP-SCD, Algorithm 5: each outer step runs coordinate descent on
 * A1^T A1 beta = bhat from beta = 0, taking at step t the coordinate of
 * largest |residual| within a uniformly random subset of size alpha_t.
 * Random subsets (ILS_SAMPLE_UNIFORM with alpha < n) need n <= 4096; the
 * greedy choice (alpha >= n) and SP-RCD (alpha = 1, ILS_SAMPLE_NORM) take any
 * n.  ILS_PREC_MIXED (with ILS_FORM_CORRECTION): A1^T A1 is formed in FP32
 * and the coordinate steps keep it and the inner residual in FP32 with FP32
 * sums; the outer residual A^T J (b - A x_k) and x stay FP64. */
int ils_rgs_solve(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                  const double* b, const double* x0, double* x, const ils_opts* opts,
                  ils_info* info /* host */);

/* ---- many right-hand sides sharing one A ---- */

/* SP (Algorithm 1) for nrhs right-hand sides B = [b_1 .. b_nrhs] (m x nrhs,
 * column-major, ldb >= p + q) with the same A: A1^T A1 and A2^T A2 are formed
 * and eliminated once, [A1^T A1 | A2^T A2 | A^T J B] -> [I | B_sp | C], and
 * every outer step X_{k+1} = B_sp X_k + C is one product over the columns
 * still iterating.  Each column has its own stop test (Sec. 5) at X_k and is
 * frozen once it passes; opts->x_ref, when given, is n x nrhs with leading
 * dimension n (the reference solution of every column).  X0 (n x nrhs,
 * ldx0 >= n) may be NULL for the zero start; X is n x nrhs with ldx >= n.
 * Only ILS_FORM_PAPER with ILS_PREC_FP64 (else ILS_ERR_ARG).
 * iters (host, nrhs entries, may be NULL) receives each column's outer count.
 * info->outer_iters, info->rr and info->rel_err are the maxima over columns.
 * Returns ILS_ERR_NO_CONVERGENCE if any column is still above tol after
 * max_outer steps (every column then holds its last iterate), and
 * ILS_ERR_NONFINITE if any column's stop quantity is not finite.  Workspace
 * grows with n * (2n + 4 nrhs) doubles. */
int ils_sp_solve_multi(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                       int64_t nrhs, const double* B, int64_t ldb, const double* X0, int64_t ldx0,
                       double* X, int64_t ldx, const ils_opts* opts, int64_t* iters /* host */,
                       ils_info* info /* host */);

/* SP on a fixed A, prepared once (Alg. 1 steps 2-5 without b): forms
 * A1^T A1 and A2^T A2 and eliminates [A1^T A1 | A2^T A2 | I] to [I | B | P]
 * (B = P A2^T A2, P = (A1^T A1)^{-1}), keeping B, P and A^T J A on the
 * device (3 n^2 doubles owned by the object).  Each later solve then costs
 * A^T J b (one product over A for all right-hand sides), c = P A^T J b and
 * its outer steps x_{k+1} = B x_k + c (Alg. 1 step 6), with the same per-
 * column stop tests and results as ils_sp_solve_multi (up to rounding in c).
 * For callers that solve many right-hand sides with one A over time, e.g.
 * with a learned warm start.  A is not copied: it must stay allocated and
 * unchanged while the object lives.  The object uses h's device, stream and
 * workspace; destroy it before h.  Errors: ILS_ERR_ARG (shapes, pointers),
 * ILS_ERR_NONFINITE (a non-finite entry of A), ILS_ERR_NOT_SPD (A1^T A1 not
 * positive definite), ILS_ERR_ALLOC; *prep is NULL on error. */
typedef struct ils_sp_prep ils_sp_prep;
int ils_sp_prepare(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                   ils_sp_prep** prep /* host out */);
/* As ils_sp_solve_multi on the prepared A (B m x nrhs, ldb >= m; X0 may be
 * NULL; X n x nrhs; ILS_FORM_PAPER, ILS_PREC_FP64 only). */
int ils_sp_prep_solve_multi(ils_sp_prep* prep, int64_t nrhs, const double* B, int64_t ldb, const double* X0,
                            int64_t ldx0, double* X, int64_t ldx, const ils_opts* opts, int64_t* iters /* host */,
                            ils_info* info /* host */);
int ils_sp_prep_destroy(ils_sp_prep* prep);

/* SP-RK-RGS (Algorithm 2) for nrhs right-hand sides B = [b_1 .. b_nrhs] (m x
 * nrhs, ldb >= p + q) with the same A and one index stream: the column draws
 * of Alg. 2 steps 8 and 10 depend only on the column norms of A1, so every
 * right-hand side uses the draws ils_rk_solve makes with the same seed, and
 * column r of X gets the iterates ils_rk_solve would give for b_r alone.
 * A block of inner steps gathers its columns of A1 once for all right-hand
 * sides, which turns the per-step inner products and updates into products
 * over the block (groups of 16 right-hand sides).  Each column has its own
 * outer stop test (Sec. 5) at x_k and inner stop test (every inner_check
 * steps, as in ils_rk_solve); a column that meets its test stops changing
 * while the others continue.  opts->x_ref, when given, is n x nrhs (leading
 * dimension n).  X0 (ldx0 >= n) may be NULL (zero start); X is n x nrhs
 * (ldx >= n).  ILS_PREC_FP64 only (else ILS_ERR_ARG); both forms.
 * iters (host, nrhs entries, may be NULL) receives each column's outer
 * count; info->outer_iters and info->rel_err are maxima over columns,
 * info->inner_iters the inner steps run.  Returns ILS_ERR_NO_CONVERGENCE if
 * any column is still above tol after max_outer outer steps.  Workspace
 * grows with (2 p + 6 n) nrhs doubles. */
int ils_rk_solve_multi(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                       int64_t nrhs, const double* B, int64_t ldb, const double* X0, int64_t ldx0,
                       double* X, int64_t ldx, const ils_opts* opts, int64_t* iters /* host */,
                       ils_info* info /* host */);

/* ---- many small problems in one launch ---- */

/* One problem of a batch; all pointers are device pointers (x0 may be NULL,
 * x_ref is required iff stop_rule == ILS_STOP_XREF). */
typedef struct {
  int64_t p, q, n, lda;
  const double* A;
  const double* b;
  const double* x0;
  const double* x_ref;
  double* x;
} ils_problem;

/* SP (Algorithm 1) on `batch` independent problems in one persistent launch:
 * each workgroup takes problems from a queue, largest n first, and runs the
 * column pass, the Gram products on the matrix cores, the block Gauss-Jordan
 * elimination and the outer steps for one problem at a time.
 * probs: host array of `batch` descriptors; infos: host array of `batch`
 * results (device_ms is the whole launch).  Supported: ILS_FORM_PAPER with
 * ILS_PREC_FP64, and ILS_FORM_CORRECTION with ILS_PREC_FP64 or ILS_PREC_MIXED
 * (FP32 Gram, FP64 elimination and residual); n <= 256 and p + q <= 4096 per
 * problem (else ILS_ERR_ARG).  The launch is captured once in a hipGraph per
 * (batch size, options) and replayed.  Returns ILS_OK, or the first non-OK
 * status among the problems in index order; x of a problem that ended in
 * ILS_ERR_NOT_SPD or ILS_ERR_NONFINITE (input) is left untouched. */
int ils_sp_solve_batched(ils_handle* h, int64_t batch, const ils_problem* probs, const ils_opts* opts,
                         ils_info* infos);

/* ---- sparse A ---- */

/* A = [A1; A2] (m = p + q rows, n columns) in CSR: rowptr (m + 1 int64),
 * colidx (nnz int32, any order within a row), val (nnz doubles), all device
 * arrays owned by the caller and read again by every solve: they must stay
 * alive and unchanged until ils_csr_destroy.  Creation checks the structure
 * (rowptr[0] = 0, rowptr[m] = nnz, non-decreasing, 0 <= colidx < n;
 * ILS_ERR_ARG otherwise) and the values (ILS_ERR_NONFINITE), and builds a
 * column-major copy (CSC, rows ascending within each column; equal rows,
 * i.e. duplicate entries, ordered by value) owned by the library.
 * Limits: 1 <= n <= 20480 (the Gram products accumulate a dense column of
 * length n on chip), m and nnz below 2^31.  The handle belongs to h's device. */
typedef struct ils_csr ils_csr;
int ils_csr_create(ils_handle* h, int64_t p, int64_t q, int64_t n, int64_t nnz, const int64_t* rowptr,
                   const int32_t* colidx, const double* val, ils_csr** A);
int ils_csr_destroy(ils_csr* A);

/* The three methods on a sparse A, with the same options and results as the
 * dense entry points: SP (Algorithm 1) with A1^T A1 and A2^T A2 formed as
 * dense n x n matrices from the sparse factors, SP-RK-RGS (Algorithm 2) on
 * the sparse columns of A1 (CSC), SP-SCD (Algorithm 5) on the dense A1^T A1.
 * The residual A^T J (b - A x) uses the CSR for A x and the CSC for A^T.
 * Only ILS_PREC_FP64 (else ILS_ERR_ARG). */
int ils_sp_solve_csr(ils_handle* h, const ils_csr* A, const double* b, const double* x0, double* x,
                     const ils_opts* opts, ils_info* info /* host */);
int ils_rk_solve_csr(ils_handle* h, const ils_csr* A, const double* b, const double* x0, double* x,
                     const ils_opts* opts, ils_info* info /* host */);
int ils_rgs_solve_csr(ils_handle* h, const ils_csr* A, const double* b, const double* x0, double* x,
                      const ils_opts* opts, ils_info* info /* host */);

/* Components on a sparse A: G = A1^T A1 (part 0) or A2^T A2 (part 1), full
 * symmetric, leading dimension ldg >= n; g = A^T J b and (colnorm2 may be
 * NULL) ||A1_(j)||^2; r = A^T J (b - A x); and a copy of the CSC arrays
 * (colptr n + 1, rowidx and val nnz, a1len n = entries of A1 per column). */
int ils_csr_gram(ils_handle* h, const ils_csr* A, int32_t part, double* G, int64_t ldg);
int ils_csr_colpass(ils_handle* h, const ils_csr* A, const double* b, double* g, double* colnorm2);
int ils_csr_residual(ils_handle* h, const ils_csr* A, const double* b, const double* x, double* r);
int ils_csr_export_csc(const ils_csr* A, int64_t* colptr, int32_t* rowidx, double* val, int32_t* a1len);

/* ---- learned warm start for a family of problems that share A ---- */

/* A three-layer perceptron d_in -> hidden -> hidden -> n (ReLU after the two
 * hidden layers, linear output) maps rows in_rows[0 .. d_in) of b to an
 * initial value x0 for the SP iteration; SP converges from any x0 (Thm. 2.1),
 * so the network changes only the number of outer steps and the zero start
 * stays the fallback.  Products run in bf16 on the matrix cores with FP32
 * accumulation; master weights, Adam moments and the loss are FP32.  Inputs
 * and targets are standardised per feature with the statistics of the last
 * training set (identity until the first ils_ws_train).
 * theta = [W1, b1, W2, b2, W3, b3], W_l row-major (d_l x d_{l-1}).
 * All arrays are device arrays unless marked host. */
typedef struct ils_ws ils_ws;

/* in_rows: host, d_in row indices in [0, m).  Weights ~ N(0, 2 / fan_in)
 * from Philox4x64-10 keyed by seed, biases 0.  The network belongs to h's
 * device and stream; destroy it before h. */
int ils_ws_create(ils_handle* h, int64_t m, int64_t n, int64_t d_in, const int64_t* in_rows, int64_t hidden,
                  uint64_t seed, ils_ws** net);
int ils_ws_destroy(ils_ws* net);

/* Train on N pairs (columns of B, m x N, ldb >= m; columns of X, n x N,
 * ldx >= n) for `epochs` passes in shuffled mini-batches of `batch` samples,
 * minimising the mean squared error of the standardised output with Adam
 * (lr, beta1 0.9, beta2 0.999, eps 1e-8).  *final_loss (host, may be NULL):
 * mean loss over the last epoch.  Returns ILS_ERR_NONFINITE if it diverges. */
int ils_ws_train(ils_ws* net, int64_t N, const double* B, int64_t ldb, const double* X, int64_t ldx,
                 int32_t epochs, int64_t batch, double lr, double* final_loss /* host */);

/* X0 (n x N, ldx0 >= n) = network estimate for each column of B. */
int ils_ws_infer(ils_ws* net, int64_t N, const double* B, int64_t ldb, double* X0, int64_t ldx0);

/* Save / load dimensions, input rows, standardisation, weights and Adam state
 * (host file path).  ils_ws_load needs a network of the same dimensions. */
int ils_ws_save(ils_ws* net, const char* path);
int ils_ws_load(ils_ws* net, const char* path);

/* Check entry points on standardised data (FP32, N columns; U is rounded to
 * bf16 as in training): number of parameters (host out), parameter copy-out
 * and copy-in (copy-in also resets the Adam state), the network output
 * Y (n x N), the loss gradient (grad: FP32, nparams; *loss host), and one
 * Adam step with a given gradient. */
int ils_ws_nparams(const ils_ws* net, int64_t* nparams /* host */);
int ils_ws_get_params(ils_ws* net, float* theta);
int ils_ws_set_params(ils_ws* net, const float* theta);
int ils_ws_forward(ils_ws* net, int64_t N, const float* U, float* Y);
int ils_ws_grad(ils_ws* net, int64_t N, const float* U, const float* T, float* grad, double* loss /* host */);
int ils_ws_adam(ils_ws* net, const float* grad, double lr);

/* ---- component entry points (used for parity checks of single steps) ---- */

/* G = A[r0:r1, :]^T A[r0:r1, :] (Alg. 1 steps 2-3), full symmetric n x n,
 * column-major with leading dimension ldg >= n.  precision ILS_PREC_MIXED
 * rounds A to FP32 and accumulates in FP32 (result widened to FP64). */
int ils_gram(ils_handle* h, int64_t r0, int64_t r1, int64_t n, const double* A, int64_t lda,
             double* G, int64_t ldg, int32_t precision);

/* G = A^T J B = A1^T B1 - A2^T B2 for many right-hand sides at once (the
 * A^T J b of Alg. 1 step 4 for every column of B; p + q rows, A m x n with
 * lda >= m, B m x nrhs with ldb >= m, G n x nrhs column-major with
 * ldg >= n; FP64).  For m >= 2048 with 16-byte aligned A and B and even lda,
 * ldb it runs on the resident per-XCD kernel of the Gram products
 * (rectangular 64 x 64 tiles, the two signs as two row parts subtracted in
 * the reduction), otherwise on the tiled product.  Waits for the result. */
int ils_atjb(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda, int64_t nrhs,
             const double* B, int64_t ldb, double* G, int64_t ldg);

/* g = A^T J b = A1^T b1 - A2^T b2 and c_j = ||A1_(j)||^2 (Alg. 1 step 4,
 * Alg. 2 steps 3, 8, 10). */
int ils_colpass(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                const double* b, double* g, double* colnorm2);

/* r = A^T J (b - A x), the residual of the normal equation (eq. Sec12). */
int ils_residual(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                 const double* b, const double* x, double* r);

/* ils_residual for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same r = A^T J (b - A x) with the default launch choice (the same bits
 * as ils_residual unless the tuning table holds a residual entry for the
 * shape), but its workspace is a fixed device array of 8 MiB (2^20 doubles) that the
 * library holds on each device until the process ends, and the call
 * allocates nothing.  It returns once the work is queued on the handle's
 * stream (r is ready when that stream's earlier work is done); it does not
 * wait.  The workspace needed is (p + q) + 256 n doubles for n <= 1024 and
 * (groups + 1)(p + q) doubles above (groups = the column groups of the
 * two-pass residual, at most ceil(n / 32)); a size that needs more than
 * 2^20 doubles returns ILS_ERR_ARG, as do the argument errors of
 * ils_residual and a handle on device ordinal 64 or above.  Every call on a
 * device shares that device's array: calls that overlap in time on one
 * device (other streams, other handles, other host threads) race and must be
 * ordered by the caller; calls queued on one stream are ordered by it.
 * Nothing in the array needs to start at zero. */
int ils_residual_noalloc(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                         const double* b, const double* x, double* r);

/* X = G^{-1} R for SPD G (n x n, ldg) and R (n x nrhs, ldr), by the block
 * Gauss-Jordan elimination used inside ils_sp_solve.  Returns
 * ILS_ERR_NOT_SPD if a pivot block is not positive definite. */
int ils_spd_solve(ils_handle* h, int64_t n, int64_t nrhs, const double* G, int64_t ldg,
                  const double* R, int64_t ldr, double* X, int64_t ldx);

/* Index streams of the randomized inner loops for outer step `outer`,
 * inner steps [t0, t0 + count): j1[i], j2[i] of SP-RK-RGS drawn with
 * probability weight_j / sum(weight) (weights: device, n), and for SP-SCD
 * alpha[i] and the bitmask of tau_t (member: count x ceil(n/32) uint32, bit s
 * of word s/32 set iff s is in the subset).  Outputs are device arrays. */
int ils_rk_indices(ils_handle* h, uint64_t seed, uint64_t outer, int64_t t0, int64_t count,
                   const double* weights, int64_t n, int32_t* j1, int32_t* j2);
int ils_scd_subsets(ils_handle* h, uint64_t seed, uint64_t outer, int64_t t0, int64_t count,
                    int64_t n, int64_t alpha_opt, int32_t* alpha, uint32_t* member);

/* ---- autotuning ---- */

enum { ILS_TUNE_GRAM = 0, ILS_TUNE_BATCHED = 1, ILS_TUNE_RESIDUAL = 2 };
enum { ILS_GRAM_SPLITK = 0, ILS_GRAM_PERSISTENT = 1 };
enum { ILS_BATCH_LARGEST_FIRST = 0, ILS_BATCH_AS_GIVEN = 1 };
enum { ILS_RESID_AUTO = 0, ILS_RESID_TWO_PASS = 1 };
/* One launch choice; the fields mean, per kernel:
 *   ILS_TUNE_GRAM     n columns, K rows; tile 64 or 128; workgroups aimed at
 *                     (ILS_GRAM_SPLITK, sets the K-split) or resident per CU
 *                     (ILS_GRAM_PERSISTENT; under ILS_PREC_MIXED it first
 *                     copies the rows to FP32 and reads the copy); kind
 *                     ILS_GRAM_*.
 *   ILS_TUNE_BATCHED  n = largest n of the batch, K = batch size; tile = rows
 *                     of A per LDS stage of the Gram products (16, 32, 64);
 *                     workgroups = resident per CU (1 or 2); kind = order the
 *                     problems are taken in (ILS_BATCH_*); reserved = form.
 *   ILS_TUNE_RESIDUAL n columns, K = p + q rows; tile 16 (rows per block);
 *                     workgroups of the one-pass kernel; kind ILS_RESID_*
 *                     (ILS_RESID_AUTO: one pass over A for n <= 1024). */
typedef struct {
  int32_t kernel;       /* ILS_TUNE_* */
  int32_t precision;    /* ILS_PREC_* */
  int64_t n, K;         /* shape the sweep ran on */
  int32_t tile;
  int32_t workgroups;
  double ms;            /* mean time of one launch */
  int32_t kind;
  int32_t reserved;
} ils_tune_entry;

/* Time every launch configuration of the Gram kernel (split-K: tile edge
 * 64 / 128 x 256 .. 8192 workgroups; the persistent kind, used where the
 * operand columns are 16-byte aligned: FP64 A with an even lda, or under
 * ILS_PREC_MIXED an FP32 copy of the rows made by the launch) on
 * G = A[0:K, :]^T A[0:K, :] (reps launches each,
 * after one warm-up; the matrix is only read) and keep the fastest for the
 * bucket (precision, ceil(log2 n), ceil(log2 K)) in the process-wide table
 * that all Gram launches consult (every solver, every handle).  *best (host,
 * may be NULL) receives the choice.  Results of later solves differ from the
 * default configuration only by the order of the K-split additions. */
int ils_tune_gram(ils_handle* h, int64_t K, int64_t n, const double* A, int64_t lda, int32_t precision,
                  int32_t reps, ils_tune_entry* best /* host */);
/* The batched solver's launch choices (Gram stage rows 16 / 32 / 64 x 1 or 2
 * resident workgroups per CU x largest-first or given order), each timed on
 * the caller's batch with ils_sp_solve_batched's options (one warm-up and
 * `reps` timed launches; every launch solves the batch, so each problem's x
 * receives its solution); the fastest is kept for the bucket (precision,
 * form, ceil(log2 largest n), ceil(log2 batch)).  Results of later batched
 * solves differ from other choices only in the order of the Gram sums. */
int ils_tune_batched(ils_handle* h, int64_t batch, const ils_problem* probs, const ils_opts* opts, int32_t reps,
                     ils_tune_entry* best /* host */);
/* The residual A^T J (b - A x)'s launch choices (one pass over A with 128,
 * 256, 512 or 1024 workgroups for n <= 1024; two passes), timed on the
 * caller's A, b, x (only read); the fastest is kept for the bucket
 * (ceil(log2 n), ceil(log2 (p + q))). */
int ils_tune_residual(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                      const double* b, const double* x, int32_t reps, ils_tune_entry* best /* host */);
/* Save / load the table as JSON (host path); load adds to the table and
 * rejects malformed files with ILS_ERR_ARG.  Clear restores the defaults. */
int ils_tune_save(const char* path);
int ils_tune_load(const char* path);
int ils_tune_clear(void);

/* ---- instrumentation ---- */

/* Phase timing of ils_sp_solve: the library records HIP events on the
 * handle's stream, between the phases of each solve (ILS_PROFILE_PHASES) or
 * only around the main Gram kernel (ILS_PROFILE_GRAM).  Kernel work is
 * unchanged, but each event costs a few microseconds of device time, so the
 * second mode is the one to keep on while timing whole solves.  Returns
 * ILS_ERR_ARG for another mode. */
enum {
  ILS_PROFILE_OFF = 0,
  ILS_PROFILE_PHASES = 1,
  ILS_PROFILE_GRAM = 2
};
int ils_set_profiling(ils_handle* h, int mode);

/* Durations in ms of the phases of the last profiled ils_sp_solve, written
 * to ms[0 .. count-1] (host; under ILS_PROFILE_GRAM only [1] is measured and
 * the others are NaN): [0] solve start to the main Gram kernel (nothing:
 * that launch is queued first), [1] main Gram kernel (dense paper form:
 * A1^T A1 and A2^T A2 with the border columns b1, b2 in one launch;
 * otherwise A1^T A1), [2] its split-K reduction, the loop-state reset, the
 * column pass (correction form, sparse A) and the norms, [3] the other Gram product if separate and right-hand
 * side assembly, [4] block Gauss-Jordan, [5] iteration matrix layout and
 * start vector, [6] outer iterations (including the host's polls of the stop
 * flag).
 * Returns the number of phases written, or a negative ils_status
 * (ILS_ERR_ARG when profiling is off). */
int ils_get_phase_times(ils_handle* h, double* ms, int count);

#ifdef __cplusplus
}
#endif
#endif
