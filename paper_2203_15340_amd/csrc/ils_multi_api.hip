// ils_multi_api.hip -- SP (Algorithm 1) for many right-hand sides that share
// one A: the Gram products and the elimination are done once, then every
// outer step is one matrix product over all live right-hand sides.
//
// W = [A1^T A1 | A2^T A2 | A^T J B] is reduced by block Gauss-Jordan to
// [I | B_sp | C] (B_sp = P A2^T A2, C = P A^T J B with P = (A1^T A1)^{-1},
// Alg. 1 steps 2-5), and X_{k+1} = B_sp X_k + C (Alg. 1 step 6) runs as
// C = X^T Y products with X = B_sp^T.  Each column has its own stop test at
// X_k (Sec. 5); a column that meets it is frozen and keeps its iterate.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ils_common.hpp"
#include "ils_runtime.hpp"

using namespace ils;

#define HIPCHK(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return ILS_ERR_HIP; \
  } while (0)

static int fail_multi(ils_info* info, int st) {
  if (info) {
    memset(info, 0, sizeof(*info));
    info->status = st;
    info->rr = NAN;
    info->rel_err = -1.0;
  }
  return st;
}

extern "C" int ils_sp_solve_multi(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A,
                                  int64_t lda, int64_t nrhs, const double* B, int64_t ldb,
                                  const double* X0, int64_t ldx0, double* X, int64_t ldx,
                                  const ils_opts* o, int64_t* iters_out, ils_info* info) {
  if (!h) return fail_multi(info, ILS_ERR_ARG);
  int st = check_problem(p, q, n, A, lda, B, X, o);
  if (st != ILS_OK) return fail_multi(info, st);
  const int64_t m = p + q;
  if (nrhs < 1 || nrhs > ((int64_t)1 << 24) || ldb < m || ldx < n || (X0 && ldx0 < n))
    return fail_multi(info, ILS_ERR_ARG);
  if (o->form != ILS_FORM_PAPER || o->precision != ILS_PREC_FP64) return fail_multi(info, ILS_ERR_ARG);
  if (hipSetDevice(h->device) != hipSuccess) return fail_multi(info, ILS_ERR_HIP);
  hipStream_t s = h->stream;
  const bool rr = o->stop_rule == ILS_STOP_RR;
  const bool fixed = o->stop_rule == ILS_STOP_FIXED;
  const int64_t ldw = n;
  double *W, *Gm = nullptr, *Xa, *Xb, *R = nullptr, *H = nullptr, *metric, *den, *Bt, *dinv;
  int* act;
  int64_t* iters;
  void* part;
  const size_t part_bytes = std::max(gram_partials_size(n, p), gram_partials_size(n, q)) * sizeof(double);
  const size_t nN = sizeof(double) * (size_t)n * (size_t)nrhs;
  if ((st = h->need(kBufW, sizeof(double) * ldw * (2 * n + nrhs), (void**)&W)) ||
      (rr && (st = h->need(kBufMG, nN, (void**)&Gm))) ||
      (rr && (st = h->need(kBufMR, nN, (void**)&R))) ||
      (rr && (st = h->need(kBufH, sizeof(double) * n * n, (void**)&H))) ||
      (st = h->need(kBufMX0, nN, (void**)&Xa)) || (st = h->need(kBufMX1, nN, (void**)&Xb)) ||
      (st = h->need(kBufMAct, sizeof(int) * nrhs, (void**)&act)) ||
      (st = h->need(kBufMIters, sizeof(int64_t) * nrhs, (void**)&iters)) ||
      (st = h->need(kBufMMetric, sizeof(double) * nrhs, (void**)&metric)) ||
      (st = h->need(kBufMDen, sizeof(double) * nrhs, (void**)&den)) ||
      (st = h->need(kBufMBt, sizeof(double) * n * n, (void**)&Bt)) ||
      (st = h->need(kBufPart, part_bytes, &part)) ||
      (st = h->need(kBufDinv, gj_scratch_bytes(n, 2 * n + nrhs), (void**)&dinv)))
    return fail_multi(info, st);

  LoopState* ds = h->st;
  HIPCHK(hipMemsetAsync(ds, 0, sizeof(LoopState), s));
  if (h->timing()) HIPCHK(hipEventRecord(h->ev0, s));
  launch_gram_f64(s, p, n, A, lda, (double*)part, W, ldw);
  launch_gram_f64(s, q, n, A + p, lda, (double*)part, W + n * ldw, ldw);
  if (rr) launch_sub(s, n, W, ldw, W + n * ldw, ldw, H, n);
  // A^T J B: rows p.. of B enter negated (J = diag(I_p, -I_q))
  GemmTnArgs gb = {};
  gb.M = n;
  gb.N = nrhs;
  gb.K = m;
  gb.X = A;
  gb.ldx = lda;
  gb.Y = B;
  gb.ldy = ldb;
  gb.kneg = p;
  gb.alpha = 1.0;
  gb.beta = 0.0;
  gb.C = rr ? Gm : W + 2 * n * ldw;
  gb.ldc = rr ? n : ldw;
  launch_gemm_tn(s, gb);
  if (rr) {
    launch_mat_copy(s, n, nrhs, Gm, n, W + 2 * n * ldw, ldw);
    launch_colnorm2(s, n, nrhs, Gm, n, den);
  } else if (o->stop_rule == ILS_STOP_XREF) {
    launch_colnorm2(s, n, nrhs, o->x_ref, n, den);
  }
  launch_gj(s, n, n + nrhs, W, ldw, dinv, &ds->bits);
  launch_transpose(s, n, n, W + n * ldw, ldw, Bt, n);
  launch_mat_copy(s, n, nrhs, X0, ldx0, Xa, n);
  launch_fill_int(s, nrhs, 1, act);

  MultiMetricArgs ma = {};
  ma.n = n;
  ma.N = nrhs;
  ma.V = rr ? R : Xa;
  ma.ldv = n;
  ma.Xref = o->x_ref;
  ma.ldr = n;
  ma.den2 = den;
  ma.stop_rule = o->stop_rule;
  ma.tol = o->tol;
  ma.active = act;
  ma.iters = iters;
  ma.metric = metric;
  ma.nactive = &ds->nactive;
  ma.bits = &ds->bits;

  GemmTnArgs gr = {};  // R = H X_k - G (RR test)
  gr.M = n;
  gr.N = nrhs;
  gr.K = n;
  gr.X = H;
  gr.ldx = n;
  gr.ldy = n;
  gr.kneg = n;
  gr.alpha = 1.0;
  gr.beta = -1.0;
  gr.C0 = Gm;
  gr.ldc0 = n;
  gr.C = R;
  gr.ldc = n;
  gr.active = act;
  GemmTnArgs gu = {};  // X_{k+1} = B_sp X_k + C
  gu.M = n;
  gu.N = nrhs;
  gu.K = n;
  gu.X = Bt;
  gu.ldx = n;
  gu.ldy = n;
  gu.kneg = n;
  gu.alpha = 1.0;
  gu.beta = 1.0;
  gu.C0 = W + 2 * n * ldw;
  gu.ldc0 = ldw;
  gu.ldc = n;
  gu.active = act;
  gu.ldkeep = n;

  double* cur = Xa;
  double* nxt = Xb;
  int64_t k = 0;
  int status = ILS_OK;
  HIPCHK(hipGetLastError());
  for (;; ++k) {
    if (!fixed) {
      if (rr) {
        gr.Y = cur;
        launch_gemm_tn(s, gr);
      }
      ma.V = rr ? R : cur;
      HIPCHK(hipMemsetAsync(&ds->nactive, 0, sizeof(int), s));
      launch_multi_metric(s, ma, k);
    }
    if (!fixed || k == 0) {
      if (h->timing()) HIPCHK(hipEventRecord(h->ev1, s));
      if ((st = read_state(h))) return fail_multi(info, st);
      const LoopState& hs = *h->st_host;
      if (hs.bits & kBitNotSpd) return fail_multi(info, ILS_ERR_NOT_SPD);
      if (hs.bits & kBitStall) return fail_multi(info, ILS_ERR_HIP);
      if (hs.bits & kBitNonfinite) {
        status = ILS_ERR_NONFINITE;
        break;
      }
      if (!fixed && hs.nactive == 0) break;
    }
    if (k == o->max_outer) {
      if (!fixed) status = ILS_ERR_NO_CONVERGENCE;
      break;
    }
    gu.Y = cur;
    gu.C = nxt;
    gu.keep = cur;
    launch_gemm_tn(s, gu);
    std::swap(cur, nxt);
  }
  launch_mat_copy(s, n, nrhs, cur, n, X, ldx);
  if (h->timing()) HIPCHK(hipEventRecord(h->ev1, s));
  HIPCHK(hipGetLastError());

  std::vector<int> hact(nrhs);
  std::vector<int64_t> hit(nrhs, 0);
  std::vector<double> hmet(nrhs, 0.0);
  HIPCHK(hipMemcpyAsync(hact.data(), act, sizeof(int) * nrhs, hipMemcpyDeviceToHost, s));
  if (!fixed) {
    HIPCHK(hipMemcpyAsync(hit.data(), iters, sizeof(int64_t) * nrhs, hipMemcpyDeviceToHost, s));
  }
  if (o->x_ref) {  // relative error of every column at its returned iterate
    MultiMetricArgs mr = ma;
    mr.V = cur;
    mr.stop_rule = ILS_STOP_XREF;
    mr.report = 1;
    if (o->stop_rule != ILS_STOP_XREF) {
      mr.den2 = den;
      launch_colnorm2(s, n, nrhs, o->x_ref, n, den);
    }
    mr.metric = metric;
    std::vector<double> relerr(nrhs);
    if (rr) {
      HIPCHK(hipMemcpyAsync(hmet.data(), metric, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    }
    launch_multi_metric(s, mr, k);
    HIPCHK(hipMemcpyAsync(relerr.data(), metric, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double worst = 0.0;
    for (double v : relerr) worst = std::max(worst, v);
    if (info) info->rel_err = worst;
  } else {
    if (rr) {
      HIPCHK(hipMemcpyAsync(hmet.data(), metric, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (info) info->rel_err = -1.0;
  }
  int64_t worst_k = 0;
  double worst_rr = 0.0;
  for (int64_t j = 0; j < nrhs; ++j) {
    if (fixed || hact[j]) hit[j] = k;
    worst_k = std::max(worst_k, hit[j]);
    worst_rr = std::max(worst_rr, hmet[j]);
  }
  if (iters_out) memcpy(iters_out, hit.data(), sizeof(int64_t) * nrhs);
  if (info) {
    info->status = status;
    info->pad = 0;
    info->outer_iters = worst_k;
    info->inner_iters = 0;
    info->rr = rr ? worst_rr : NAN;
    float ms = 0.0f;
    info->device_ms = (h->timing() && hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) ? ms : 0.0;
  }
  return status;
}
