// ils_rand_api.hip -- drivers of SP-RK-RGS (Algorithm 2) and SP-SCD
// (Algorithm 5) behind include/ils.h.
//
// Outer step k: stop test at x_k, right-hand side (A2^T A2 x_k + A^T J b, or
// the residual A^T J (b - A x_k) in the correction form), then the inner loop
// in blocks of steps: the block's random draws are made for all its steps at
// once on the whole GPU, then one workgroup runs the dependent chain.  The
// host reads the inner stop flag once per block.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "ils_common.hpp"
#include "ils_runtime.hpp"
#include "k_rand.hpp"

using namespace ils;

#define HIPCHK(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return ILS_ERR_HIP; \
  } while (0)

static int fail_info(ils_info* info, int st) {
  if (info) {
    memset(info, 0, sizeof(*info));
    info->status = st;
    info->rr = NAN;
    info->rel_err = -1.0;
  }
  return st;
}

__global__ void k_check0(const double* tn2, double itol2, int* inner_done) {
  if (threadIdx.x == 0 && *tn2 <= itol2 * (*tn2)) *inner_done = 1;
}

static double default_itol(const ils_opts* o) {
  if (o->inner_tol > 0.0) return o->inner_tol;
  return o->form == ILS_FORM_CORRECTION ? 1e-2 : 1e-8;
}

namespace {
struct Common {
  double *g, *xb0, *xb1, *tgt, *rk, *tv, *part, *G2;
};
}  // namespace

// Setup shared by both methods: A^T J b, norms for the stop test, A2^T A2
// (paper form), the start vector.
static int common_setup(ils_handle* h, const MatOp& M, const double* b, const double* x0, const ils_opts* o,
                        double* cn, Common& c) {
  hipStream_t s = h->stream;
  const int64_t n = M.n;
  const int64_t m = M.p + M.q;
  int st;
  const bool paper = o->form == ILS_FORM_PAPER;
  if ((st = h->need(kBufG, sizeof(double) * n, (void**)&c.g)) ||
      (st = h->need(kBufX0, sizeof(double) * n, (void**)&c.xb0)) ||
      (st = h->need(kBufX1, sizeof(double) * n, (void**)&c.xb1)) ||
      (st = h->need(kBufSPart, sizeof(double) * n, (void**)&c.tgt)) ||
      (st = h->need(kBufR, sizeof(double) * n, (void**)&c.rk)) ||
      (st = h->need(kBufT, sizeof(double) * residual_scratch(m, n), (void**)&c.tv)) ||
      (st = h->need(kBufPart, mat_gram_partials(M) * sizeof(double), (void**)&c.part)) ||
      (paper && (st = h->need(kBufG2, sizeof(double) * n * n, (void**)&c.G2))))
    return st;
  if (!paper) c.G2 = nullptr;
  HIPCHK(hipMemsetAsync(h->st, 0, sizeof(LoopState), s));
  if (h->timing()) HIPCHK(hipEventRecord(h->ev0, s));
  mat_colpass(s, M, b, c.g, cn, &h->st->bits);
  if (o->stop_rule == ILS_STOP_RR) launch_norm2(s, n, c.g, &h->st->scal[0]);
  if (o->stop_rule == ILS_STOP_XREF) launch_norm2(s, n, o->x_ref, &h->st->scal[1]);
  if (paper) mat_gram(s, M, 1, ILS_PREC_FP64, c.part, c.G2, n);
  launch_fill_vec(s, n, x0, c.xb0);
  return ILS_OK;
}

// Stop test at x_k; returns 1 when the outer loop is over.
static int outer_begin(ils_handle* h, const MatOp& M, const double* b, const ils_opts* o, Common& c, int64_t k,
                       int* over) {
  hipStream_t s = h->stream;
  const int64_t n = M.n;
  const double* xk = (k & 1) ? c.xb1 : c.xb0;
  const bool paper = o->form == ILS_FORM_PAPER;
  if (o->stop_rule == ILS_STOP_RR || !paper)
    mat_residual(s, M, b, xk, c.tv, c.rk, nullptr);
  launch_outer_test(s, n, xk, o->x_ref, c.rk, o->stop_rule, o->tol, k, o->max_outer, h->st);
  if (paper) launch_symv_add(s, n, c.G2, n, xk, c.g, c.tgt, &h->st->done);
  else launch_fill_vec(s, n, c.rk, c.tgt);
  launch_norm2(s, n, c.tgt, &h->st->scal[2]);
  HIPCHK(hipMemsetAsync(&h->st->inner_done, 0, sizeof(int), s));
  HIPCHK(hipMemsetAsync(&h->st->steps, 0, sizeof(int64_t), s));
  int rs = read_state(h);
  if (rs) return rs;
  *over = h->st_host->done || h->st_host->bits;
  return ILS_OK;
}

static int finish(ils_handle* h, int64_t n, double* x, const ils_opts* o, Common& c, int64_t inner_total,
                  ils_info* info) {
  if (h->timing()) HIPCHK(hipEventRecord(h->ev1, h->stream));
  int st = read_state(h);
  if (st) return fail_info(info, st);
  const LoopState& hs = *h->st_host;
  st = setup_status(hs);
  if (st != ILS_OK) return fail_info(info, st);
  if (!hs.done) return fail_info(info, ILS_ERR_HIP);
  HIPCHK(hipMemcpyAsync(x, (hs.iters & 1) ? c.xb1 : c.xb0, sizeof(double) * n, hipMemcpyDeviceToDevice,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return finish_info(h, n, x, o, hs.status, hs.iters, inner_total, hs.metric, info);
}

// ------------------------------------------------------------------ SP-RK-RGS
int ils::rk_solve_op(ils_handle* h, const MatOp& M, const double* b, const double* x0, double* x,
                     const ils_opts* o, ils_info* info) {
  if (!h) return fail_info(info, ILS_ERR_ARG);
  const int64_t p = M.p, n = M.n;
  int st = check_op(M, b, x, o);
  if (st != ILS_OK) return fail_info(info, st);
  if (hipSetDevice(h->device) != hipSuccess) return fail_info(info, ILS_ERR_HIP);
  hipStream_t s = h->stream;
  const bool fixed = o->stop_rule == ILS_STOP_FIXED;
  const int64_t max_inner = o->max_inner >= 0 ? o->max_inner : 1000 * n;
  const int64_t check = o->inner_check > 0 ? o->inner_check : n;
  const int64_t chunk = fixed ? 4096 : check;
  const double itol = default_itol(o);
  Common c;
  double *cn, *prefix, *w, *sv, *v, *z, *res2;
  int* jj;
  if ((st = h->need(kBufCn, sizeof(double) * n, (void**)&cn)) ||
      (st = h->need(kBufPrefix, sizeof(double) * n, (void**)&prefix)) ||
      (st = h->need(kBufW1, sizeof(double) * p, (void**)&w)) ||
      (st = h->need(kBufS1, sizeof(double) * p, (void**)&sv)) ||
      (st = h->need(kBufA1f, sizeof(double) * p, (void**)&v)) ||
      (st = h->need(kBufZ, sizeof(double) * n, (void**)&z)) ||
      (st = h->need(kBufH, sizeof(double) * n, (void**)&res2)) ||
      (st = h->need(kBufIdx, sizeof(int) * 2 * chunk, (void**)&jj)))
    return fail_info(info, st);
  // mixed precision: FP32 copy of A1; w and s are FP32 (same slots, half used)
  const bool mixed = o->precision == ILS_PREC_MIXED;
  float* a1f = nullptr;
  if (mixed && (st = h->need(kBufA1f32, sizeof(float) * p * n, (void**)&a1f))) return fail_info(info, st);
  const size_t wbytes = (mixed ? sizeof(float) : sizeof(double)) * p;
  // dense A: inner steps in blocks over the whole GPU; sparse A: one workgroup
  double* rkb = nullptr;
  if (!M.sp && (st = h->need(kBufRkb, sizeof(double) * rk_block_scratch(p), (void**)&rkb))) return fail_info(info, st);
  if ((st = common_setup(h, M, b, x0, o, cn, c))) return fail_info(info, st);
  if (mixed) launch_to_f32(s, p, n, M.A, M.lda, a1f);
  launch_zero_col_check(s, n, cn, &h->st->bits);  // a zero column of A1: rank(A1) < n
  launch_prefix(s, n, cn, 1, prefix);
  int64_t inner_total = 0;
  for (int64_t k = 0;; ++k) {
    int over = 0;
    if ((st = outer_begin(h, M, b, o, c, k, &over))) return fail_info(info, st);
    if (over) break;
    HIPCHK(hipMemsetAsync(w, 0, wbytes, s));
    HIPCHK(hipMemsetAsync(sv, 0, wbytes, s));
    HIPCHK(hipMemsetAsync(z, 0, sizeof(double) * n, s));
    if (!fixed) hipLaunchKernelGGL(k_check0, dim3(1), dim3(64), 0, s, &h->st->scal[2], itol * itol, &h->st->inner_done);
    int64_t t = 0;
    if (!fixed) {
      if ((st = read_state(h))) return fail_info(info, st);
    }
    while (t < max_inner && !(!fixed && h->st_host->inner_done)) {
      const int64_t cnt = std::min(chunk, max_inner - t);
      launch_rk_draw(s, o->seed, (uint64_t)k + o->stream_offset, t, cnt, prefix, n, jj, jj + chunk);
      if (mixed)
        launch_rk_blocks_f32(s, a1f, p, p, c.tgt, cn, jj, jj + chunk, cnt, (float*)w, (float*)sv, z, rkb,
                             &h->st->arrive3, &h->st->inner_done, &h->st->done);
      else if (!M.sp)
        launch_rk_blocks(s, M.A, M.lda, p, c.tgt, cn, jj, jj + chunk, cnt, w, sv, z, rkb, &h->st->arrive3,
                         &h->st->inner_done, &h->st->done);
      else
        mat_rk_inner(s, M, c.tgt, cn, jj, jj + chunk, cnt, w, sv, z, &h->st->inner_done, &h->st->done);
      t += cnt;
      if (!fixed && t % check == 0) {
        if (mixed)
          launch_rk_check_f32(s, M.A, M.lda, p, n, (const float*)w, (const float*)sv, v, c.tgt, res2,
                              itol * itol, &h->st->scal[2], &h->st->inner_done, &h->st->arrive2, &h->st->done);
        else
          mat_rk_check(s, M, w, sv, v, c.tgt, res2, itol * itol, &h->st->scal[2], &h->st->inner_done,
                       &h->st->arrive2, &h->st->done);
        if ((st = read_state(h))) return fail_info(info, st);
      }
    }
    inner_total += t;
    launch_outer_update(s, n, (k & 1) ? c.xb1 : c.xb0, z, o->form == ILS_FORM_CORRECTION,
                        (k & 1) ? c.xb0 : c.xb1, k, h->st);
  }
  return finish(h, n, x, o, c, inner_total, info);
}

extern "C" int ils_rk_solve(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                            const double* b, const double* x0, double* x, const ils_opts* o, ils_info* info) {
  MatOp M;
  M.p = p;
  M.q = q;
  M.n = n;
  M.A = A;
  M.lda = lda;
  return rk_solve_op(h, M, b, x0, x, o, info);
}

// ------------------------------------------------------------------ SP-SCD
int ils::rgs_solve_op(ils_handle* h, const MatOp& M, const double* b, const double* x0, double* x,
                      const ils_opts* o, ils_info* info) {
  if (!h) return fail_info(info, ILS_ERR_ARG);
  const int64_t n = M.n;
  int st = check_op(M, b, x, o);
  if (st == ILS_OK && o->sampling == ILS_SAMPLE_NORM && o->alpha != 1) st = ILS_ERR_ARG;
  if (st == ILS_OK && o->sampling == ILS_SAMPLE_UNIFORM && !(o->alpha >= n) && n > kScdMaxN)
    st = ILS_ERR_ARG;
  if (st != ILS_OK) return fail_info(info, st);
  if (hipSetDevice(h->device) != hipSuccess) return fail_info(info, ILS_ERR_HIP);
  hipStream_t s = h->stream;
  const bool fixed = o->stop_rule == ILS_STOP_FIXED;
  const bool norm_mode = o->sampling == ILS_SAMPLE_NORM;
  const int64_t max_inner = o->max_inner >= 0 ? o->max_inner : 1000 * n;
  const int64_t chunk = 4096;
  const int64_t words = (n + 31) / 32;
  const double itol = default_itol(o);
  Common c;
  double *G1, *W, *diag, *prefix, *r, *beta, *dinv;
  int *alpha_buf, *jpre;
  uint32_t* mask;
  if ((st = h->need(kBufM, sizeof(double) * n * n, (void**)&G1)) ||
      (st = h->need(kBufW, sizeof(double) * n * n, (void**)&W)) ||
      (st = h->need(kBufCn, sizeof(double) * n, (void**)&diag)) ||
      (st = h->need(kBufPrefix, sizeof(double) * n, (void**)&prefix)) ||
      (st = h->need(kBufZ, sizeof(double) * n, (void**)&beta)) ||
      (st = h->need(kBufW1, sizeof(double) * n, (void**)&r)) ||
      (st = h->need(kBufIdx, sizeof(int) * 2 * chunk, (void**)&alpha_buf)) ||
      (st = h->need(kBufMask, sizeof(uint32_t) * words * chunk, (void**)&mask)) ||
      (st = h->need(kBufDinv, gj_scratch_bytes(n, n), (void**)&dinv)))
    return fail_info(info, st);
  jpre = alpha_buf + chunk;
  // mixed precision: the inner sweeps read an FP32 A1^T A1 and keep r in FP32
  const bool mixed = o->precision == ILS_PREC_MIXED;
  float *G1f = nullptr, *rf = nullptr;
  if (mixed && ((st = h->need(kBufA1f32, sizeof(float) * n * n, (void**)&G1f)) ||
                (st = h->need(kBufA1f, sizeof(float) * n, (void**)&rf))))
    return fail_info(info, st);
  if ((st = common_setup(h, M, b, x0, o, nullptr, c))) return fail_info(info, st);
  mat_gram(s, M, 0, o->precision, c.part, G1, n);
  // positive definiteness of A1^T A1 (the elimination is only a test here)
  launch_copy_cols(s, n, n, G1, n, W, n);
  launch_gj(s, n, 0, W, n, dinv, &h->st->bits);
  launch_diag(s, n, G1, n, diag);
  launch_prefix(s, n, diag, 1, prefix);
  if (mixed) launch_to_f32(s, n, n, G1, n, G1f);  // FP32 sums already: exact
  int64_t inner_total = 0;
  for (int64_t k = 0;; ++k) {
    int over = 0;
    if ((st = outer_begin(h, M, b, o, c, k, &over))) return fail_info(info, st);
    if (over) break;
    if (mixed) launch_to_f32(s, n, 1, c.tgt, n, rf);
    else launch_fill_vec(s, n, c.tgt, r);
    HIPCHK(hipMemsetAsync(beta, 0, sizeof(double) * n, s));
    int64_t t = 0;
    while (true) {
      const int64_t cnt = std::min(chunk, max_inner - t);
      launch_scd_draw(s, o->seed, (uint64_t)k + o->stream_offset, t, cnt, n, o->alpha, norm_mode, prefix,
                      alpha_buf, jpre, mask, words);
      if (mixed)
        launch_scd_inner_f32(s, G1f, n, n, rf, beta, mask, words, jpre, norm_mode, cnt, !fixed, itol * itol,
                             &h->st->scal[2], &h->st->inner_done, &h->st->steps, &h->st->done);
      else
        launch_scd_inner(s, G1, n, n, r, beta, mask, words, jpre, norm_mode, cnt, !fixed, itol * itol,
                         &h->st->scal[2], &h->st->inner_done, &h->st->steps, &h->st->done);
      t += cnt;
      if ((st = read_state(h))) return fail_info(info, st);
      if (h->st_host->inner_done || t >= max_inner || h->st_host->done) break;
    }
    inner_total += h->st_host->steps;
    launch_outer_update(s, n, (k & 1) ? c.xb1 : c.xb0, beta, o->form == ILS_FORM_CORRECTION,
                        (k & 1) ? c.xb0 : c.xb1, k, h->st);
  }
  return finish(h, n, x, o, c, inner_total, info);
}

extern "C" int ils_rgs_solve(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                             const double* b, const double* x0, double* x, const ils_opts* o, ils_info* info) {
  MatOp M;
  M.p = p;
  M.q = q;
  M.n = n;
  M.A = A;
  M.lda = lda;
  return rgs_solve_op(h, M, b, x0, x, o, info);
}

// ------------------------------------------------------------------ index streams
extern "C" int ils_rk_indices(ils_handle* h, uint64_t seed, uint64_t outer, int64_t t0, int64_t count,
                              const double* weights, int64_t n, int32_t* j1, int32_t* j2) {
  if (!h || !weights || !j1 || !j2 || n < 1 || count < 0 || t0 < 0) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  double* prefix;
  int st = h->need(kBufPrefix, sizeof(double) * n, (void**)&prefix);
  if (st) return st;
  launch_prefix(h->stream, n, weights, 1, prefix);
  launch_rk_draw(h->stream, seed, outer, t0, count, prefix, n, j1, j2);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return ILS_OK;
}

extern "C" int ils_scd_subsets(ils_handle* h, uint64_t seed, uint64_t outer, int64_t t0, int64_t count,
                               int64_t n, int64_t alpha_opt, int32_t* alpha, uint32_t* member) {
  if (!h || !alpha || !member || n < 1 || count < 0 || t0 < 0 || alpha_opt < 0) return ILS_ERR_ARG;
  if (!(alpha_opt >= n) && n > kScdMaxN) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  launch_scd_draw(h->stream, seed, outer, t0, count, n, alpha_opt, 0, nullptr, alpha, nullptr, member,
                  (n + 31) / 32);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return ILS_OK;
}
