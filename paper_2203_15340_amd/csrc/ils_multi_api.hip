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
#include <new>
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

namespace {

// Per-solve buffers of the multi-right-hand-side outer loop (handle-owned).
struct MultiBufs {
  double *Gm = nullptr, *Xa = nullptr, *Xb = nullptr, *R = nullptr, *metric = nullptr, *den = nullptr;
  int* act = nullptr;
  int64_t* iters = nullptr;
};

int multi_bufs(ils_handle* h, int64_t n, int64_t nrhs, bool need_g, bool rr, MultiBufs& b) {
  const size_t nN = sizeof(double) * (size_t)n * (size_t)nrhs;
  int st;
  if ((need_g && (st = h->need(kBufMG, nN, (void**)&b.Gm))) || (rr && (st = h->need(kBufMR, nN, (void**)&b.R))) ||
      (st = h->need(kBufMX0, nN, (void**)&b.Xa)) || (st = h->need(kBufMX1, nN, (void**)&b.Xb)) ||
      (st = h->need(kBufMAct, sizeof(int) * nrhs, (void**)&b.act)) ||
      (st = h->need(kBufMIters, sizeof(int64_t) * nrhs, (void**)&b.iters)) ||
      (st = h->need(kBufMMetric, sizeof(double) * nrhs, (void**)&b.metric)) ||
      (st = h->need(kBufMDen, sizeof(double) * nrhs, (void**)&b.den)))
    return st;
  return ILS_OK;
}

// Products that take the persistent kernel: long contractions (A^T J B over
// the rows of A), and the n x n products of the outer steps once there are
// enough tiles to fill the grid.
constexpr int64_t kAtjbPersMinRows = 2048;
constexpr int64_t kStepPersMinK = 512;
constexpr int64_t kStepPersMinTiles = 64;

bool step_pers(int64_t n, int64_t nrhs) {
  return n >= kStepPersMinK && ((n + 63) / 64) * ((nrhs + 63) / 64) >= kStepPersMinTiles;
}

// Partial-tile scratch (doubles) the products of a solve may use.
size_t atjb_partials(int64_t p, int64_t q, int64_t n, int64_t nrhs) {
  return p + q >= kAtjbPersMinRows ? gemm_tn_pers_partials(p + q, n, nrhs) : 0;
}
size_t step_partials(int64_t n, int64_t nrhs) { return step_pers(n, nrhs) ? gemm_tn_pers_partials(n, n, nrhs) : 0; }

// C = alpha X^T S Y + beta C0 on the persistent kernel where `pers` holds and
// it applies, else on the tiled product.
void gemm(hipStream_t s, const GemmTnArgs& g, bool pers, double* partials, size_t partial_doubles) {
  if (pers && partials && launch_gemm_tn_pers(s, g, partials, partial_doubles)) return;
  launch_gemm_tn(s, g);
}

// A^T J B into G (n x nrhs, ldg): rows p.. of B enter negated (J = diag(I_p, -I_q)).
void atjb(hipStream_t s, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda, int64_t nrhs,
          const double* B, int64_t ldb, double* G, int64_t ldg, double* partials, size_t partial_doubles) {
  GemmTnArgs gb = {};
  gb.M = n;
  gb.N = nrhs;
  gb.K = p + q;
  gb.X = A;
  gb.ldx = lda;
  gb.Y = B;
  gb.ldy = ldb;
  gb.kneg = p;
  gb.alpha = 1.0;
  gb.beta = 0.0;
  gb.C = G;
  gb.ldc = ldg;
  gemm(s, gb, p + q >= kAtjbPersMinRows, partials, partial_doubles);
}

// Alg. 1 step 6 for every column: X_{k+1} = B X_k + C (Bt = B^T, n x n;
// C n x nrhs, ldc), from X0 (null: zero), each column with its own stop test
// at X_k (Sec. 5: RR needs H = A^T J A and G = A^T J B in mb.Gm; XREF the
// references in o->x_ref), frozen once it passes.  The device state has been
// reset by the caller, which also holds h->ev0 when timing.
int multi_iterate(ils_handle* h, int64_t n, int64_t nrhs, const double* Bt, const double* Cm, int64_t ldc,
                  const double* H, const MultiBufs& mb, const double* X0, int64_t ldx0, double* X, int64_t ldx,
                  const ils_opts* o, int64_t* iters_out, ils_info* info, double* partials,
                  size_t partial_doubles) {
  const bool pers = step_pers(n, nrhs);
  hipStream_t s = h->stream;
  LoopState* ds = h->st;
  const bool rr = o->stop_rule == ILS_STOP_RR;
  const bool fixed = o->stop_rule == ILS_STOP_FIXED;
  int st;
  if (rr)
    launch_colnorm2(s, n, nrhs, mb.Gm, n, mb.den);
  else if (o->stop_rule == ILS_STOP_XREF)
    launch_colnorm2(s, n, nrhs, o->x_ref, n, mb.den);
  launch_mat_copy(s, n, nrhs, X0, ldx0, mb.Xa, n);
  launch_fill_int(s, nrhs, 1, mb.act);

  MultiMetricArgs ma = {};
  ma.n = n;
  ma.N = nrhs;
  ma.V = rr ? mb.R : mb.Xa;
  ma.ldv = n;
  ma.Xref = o->x_ref;
  ma.ldr = n;
  ma.den2 = mb.den;
  ma.stop_rule = o->stop_rule;
  ma.tol = o->tol;
  ma.active = mb.act;
  ma.iters = mb.iters;
  ma.metric = mb.metric;
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
  gr.C0 = mb.Gm;
  gr.ldc0 = n;
  gr.C = mb.R;
  gr.ldc = n;
  gr.active = mb.act;
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
  gu.C0 = Cm;
  gu.ldc0 = ldc;
  gu.ldc = n;
  gu.active = mb.act;
  gu.ldkeep = n;

  double* cur = mb.Xa;
  double* nxt = mb.Xb;
  int64_t k = 0;
  int status = ILS_OK;
  HIPCHK(hipGetLastError());
  for (;; ++k) {
    if (!fixed) {
      if (rr) {
        gr.Y = cur;
        gemm(s, gr, pers, partials, partial_doubles);
      }
      ma.V = rr ? mb.R : cur;
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
    gemm(s, gu, pers, partials, partial_doubles);
    std::swap(cur, nxt);
  }
  launch_mat_copy(s, n, nrhs, cur, n, X, ldx);
  if (h->timing()) HIPCHK(hipEventRecord(h->ev1, s));
  HIPCHK(hipGetLastError());

  std::vector<int> hact(nrhs);
  std::vector<int64_t> hit(nrhs, 0);
  std::vector<double> hmet(nrhs, 0.0);
  HIPCHK(hipMemcpyAsync(hact.data(), mb.act, sizeof(int) * nrhs, hipMemcpyDeviceToHost, s));
  if (!fixed) {
    HIPCHK(hipMemcpyAsync(hit.data(), mb.iters, sizeof(int64_t) * nrhs, hipMemcpyDeviceToHost, s));
  }
  if (o->x_ref) {  // relative error of every column at its returned iterate
    MultiMetricArgs mr = ma;
    mr.V = cur;
    mr.stop_rule = ILS_STOP_XREF;
    mr.report = 1;
    if (o->stop_rule != ILS_STOP_XREF) {
      mr.den2 = mb.den;
      launch_colnorm2(s, n, nrhs, o->x_ref, n, mb.den);
    }
    mr.metric = mb.metric;
    std::vector<double> relerr(nrhs);
    if (rr) {
      HIPCHK(hipMemcpyAsync(hmet.data(), mb.metric, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    }
    launch_multi_metric(s, mr, k);
    HIPCHK(hipMemcpyAsync(relerr.data(), mb.metric, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double worst = 0.0;
    for (double v : relerr) worst = std::max(worst, v);
    if (info) info->rel_err = worst;
  } else {
    if (rr) {
      HIPCHK(hipMemcpyAsync(hmet.data(), mb.metric, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
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

int check_multi(int64_t m, int64_t n, int64_t nrhs, int64_t ldb, int64_t ldx, const double* X0, int64_t ldx0,
                const ils_opts* o) {
  if (nrhs < 1 || nrhs > ((int64_t)1 << 24) || ldb < m || ldx < n || (X0 && ldx0 < n)) return ILS_ERR_ARG;
  if (o->form != ILS_FORM_PAPER || o->precision != ILS_PREC_FP64) return ILS_ERR_ARG;
  return ILS_OK;
}

}  // namespace

extern "C" int ils_atjb(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                        int64_t nrhs, const double* B, int64_t ldb, double* G, int64_t ldg) {
  const int64_t m = p + q;
  if (!h || !A || !B || !G || n < 1 || p < 0 || q < 0 || m < 1 || nrhs < 1 || lda < m || ldb < m || ldg < n)
    return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  const size_t part_doubles = atjb_partials(p, q, n, nrhs);
  void* part = nullptr;
  int st;
  if (part_doubles && (st = h->need(kBufPart, part_doubles * sizeof(double), &part))) return st;
  atjb(h->stream, p, q, n, A, lda, nrhs, B, ldb, G, ldg, (double*)part, part_doubles);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return ILS_OK;
}

extern "C" int ils_sp_solve_multi(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A,
                                  int64_t lda, int64_t nrhs, const double* B, int64_t ldb,
                                  const double* X0, int64_t ldx0, double* X, int64_t ldx,
                                  const ils_opts* o, int64_t* iters_out, ils_info* info) {
  if (!h) return fail_multi(info, ILS_ERR_ARG);
  int st = check_problem(p, q, n, A, lda, B, X, o);
  if (st != ILS_OK) return fail_multi(info, st);
  const int64_t m = p + q;
  if ((st = check_multi(m, n, nrhs, ldb, ldx, X0, ldx0, o))) return fail_multi(info, st);
  if (hipSetDevice(h->device) != hipSuccess) return fail_multi(info, ILS_ERR_HIP);
  hipStream_t s = h->stream;
  const bool rr = o->stop_rule == ILS_STOP_RR;
  const int64_t ldw = n;
  double *W, *H = nullptr, *Bt, *dinv;
  void* part;
  MultiBufs mb;
  const size_t part_doubles = std::max({gram_partials_size(n, p), gram_partials_size(n, q),
                                        atjb_partials(p, q, n, nrhs), step_partials(n, nrhs)});
  const size_t part_bytes = part_doubles * sizeof(double);
  if ((st = h->need(kBufW, sizeof(double) * ldw * (2 * n + nrhs), (void**)&W)) ||
      (st = multi_bufs(h, n, nrhs, rr, rr, mb)) ||
      (rr && (st = h->need(kBufH, sizeof(double) * n * n, (void**)&H))) ||
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
  if (rr) {
    atjb(s, p, q, n, A, lda, nrhs, B, ldb, mb.Gm, n, (double*)part, part_doubles);
    launch_mat_copy(s, n, nrhs, mb.Gm, n, W + 2 * n * ldw, ldw);
  } else {
    atjb(s, p, q, n, A, lda, nrhs, B, ldb, W + 2 * n * ldw, ldw, (double*)part, part_doubles);
  }
  // [A1^T A1 | A2^T A2 | A^T J B] -> [I | B_sp | C]
  launch_gj(s, n, n + nrhs, W, ldw, dinv, &ds->bits);
  launch_transpose(s, n, n, W + n * ldw, ldw, Bt, n);
  return multi_iterate(h, n, nrhs, Bt, W + 2 * n * ldw, ldw, H, mb, X0, ldx0, X, ldx, o, iters_out, info,
                       (double*)part, part_doubles);
}

// ------------------------------------------------------------------ prepared A
struct ils_sp_prep {
  ils_handle* h = nullptr;
  int64_t p = 0, q = 0, n = 0, lda = 0;
  const double* A = nullptr;
  double* mats = nullptr;  // device: B^T, P, H (n x n each)
  double* Bt() const { return mats; }
  double* P() const { return mats + n * n; }
  double* H() const { return mats + 2 * n * n; }
};

extern "C" int ils_sp_prepare(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                              ils_sp_prep** out) {
  if (!h || !out) return ILS_ERR_ARG;
  *out = nullptr;
  ils_opts o;
  ils_opts_default(&o);
  // check_problem wants a b and an x; A's own checks are what matter here
  int st = check_problem(p, q, n, A, lda, A, A, &o);
  if (st != ILS_OK) return st;
  if (hipSetDevice(h->device) != hipSuccess) return ILS_ERR_HIP;
  hipStream_t s = h->stream;
  const int64_t ldw = n;
  double *W, *dinv;
  void* part;
  const size_t part_bytes = std::max(gram_partials_size(n, p), gram_partials_size(n, q)) * sizeof(double);
  if ((st = h->need(kBufW, sizeof(double) * ldw * 3 * n, (void**)&W)) ||
      (st = h->need(kBufPart, part_bytes, &part)) ||
      (st = h->need(kBufDinv, gj_scratch_bytes(n, 3 * n), (void**)&dinv)))
    return st;
  ils_sp_prep* pr = new (std::nothrow) ils_sp_prep;
  if (!pr) return ILS_ERR_ALLOC;
  pr->h = h;
  pr->p = p;
  pr->q = q;
  pr->n = n;
  pr->A = A;
  pr->lda = lda;
  if (hipMalloc(&pr->mats, sizeof(double) * 3 * n * n) != hipSuccess) {
    delete pr;
    return ILS_ERR_ALLOC;
  }
  LoopState* ds = h->st;
  if (hipMemsetAsync(ds, 0, sizeof(LoopState), s) != hipSuccess) st = ILS_ERR_HIP;
  if (st == ILS_OK) {
    // [A1^T A1 | A2^T A2 | I] -> [I | B | P]  (Alg. 1 steps 2-5 without b)
    launch_gram_f64(s, p, n, A, lda, (double*)part, W, ldw);
    launch_gram_f64(s, q, n, A + p, lda, (double*)part, W + n * ldw, ldw);
    launch_sub(s, n, W, ldw, W + n * ldw, ldw, pr->H(), n);
    launch_diag_screen(s, n, W, W + n * ldw, ldw, &ds->bits);
    launch_eye(s, n, W + 2 * n * ldw, ldw);
    launch_gj(s, n, 2 * n, W, ldw, dinv, &ds->bits);
    launch_transpose(s, n, n, W + n * ldw, ldw, pr->Bt(), n);
    launch_mat_copy(s, n, n, W + 2 * n * ldw, ldw, pr->P(), n);
    if (hipGetLastError() != hipSuccess) st = ILS_ERR_HIP;
  }
  if (st == ILS_OK) st = read_state(h);
  if (st == ILS_OK) {
    const LoopState& hs = *h->st_host;
    if (hs.bits & kBitNonfinite) st = ILS_ERR_NONFINITE;
    else if (hs.bits & kBitNotSpd) st = ILS_ERR_NOT_SPD;
    else if (hs.bits & kBitStall) st = ILS_ERR_HIP;
  }
  if (st != ILS_OK) {
    (void)hipFree(pr->mats);
    delete pr;
    return st;
  }
  *out = pr;
  return ILS_OK;
}

extern "C" int ils_sp_prep_destroy(ils_sp_prep* pr) {
  if (!pr) return ILS_OK;
  if (pr->mats) {
    (void)hipSetDevice(pr->h->device);
    (void)hipStreamSynchronize(pr->h->stream);
    (void)hipFree(pr->mats);
  }
  delete pr;
  return ILS_OK;
}

extern "C" int ils_sp_prep_solve_multi(ils_sp_prep* pr, int64_t nrhs, const double* B, int64_t ldb,
                                       const double* X0, int64_t ldx0, double* X, int64_t ldx, const ils_opts* o,
                                       int64_t* iters_out, ils_info* info) {
  if (!pr || !B || !X || !o) return fail_multi(info, ILS_ERR_ARG);
  ils_handle* h = pr->h;
  const int64_t p = pr->p, q = pr->q, n = pr->n, m = p + q;
  int st = check_problem(p, q, n, pr->A, pr->lda, B, X, o);
  if (st != ILS_OK) return fail_multi(info, st);
  if ((st = check_multi(m, n, nrhs, ldb, ldx, X0, ldx0, o))) return fail_multi(info, st);
  if (hipSetDevice(h->device) != hipSuccess) return fail_multi(info, ILS_ERR_HIP);
  hipStream_t s = h->stream;
  const bool rr = o->stop_rule == ILS_STOP_RR;
  double* Cm;
  void* part = nullptr;
  MultiBufs mb;
  const size_t part_doubles = std::max({atjb_partials(p, q, n, nrhs), step_partials(n, nrhs),
                                        step_pers(n, nrhs) ? gemm_tn_pers_partials(n, n, nrhs) : (size_t)0});
  if ((st = multi_bufs(h, n, nrhs, true, rr, mb)) ||
      (st = h->need(kBufMC, sizeof(double) * (size_t)n * (size_t)nrhs, (void**)&Cm)) ||
      (part_doubles && (st = h->need(kBufPart, part_doubles * sizeof(double), &part))))
    return fail_multi(info, st);
  HIPCHK(hipMemsetAsync(h->st, 0, sizeof(LoopState), s));
  if (h->timing()) HIPCHK(hipEventRecord(h->ev0, s));
  atjb(s, p, q, n, pr->A, pr->lda, nrhs, B, ldb, mb.Gm, n, (double*)part, part_doubles);
  GemmTnArgs gc = {};  // C = P A^T J B (P symmetric, so P^T Y = P Y)
  gc.M = n;
  gc.N = nrhs;
  gc.K = n;
  gc.X = pr->P();
  gc.ldx = n;
  gc.Y = mb.Gm;
  gc.ldy = n;
  gc.kneg = n;
  gc.alpha = 1.0;
  gc.beta = 0.0;
  gc.C = Cm;
  gc.ldc = n;
  gemm(s, gc, step_pers(n, nrhs), (double*)part, part_doubles);
  return multi_iterate(h, n, nrhs, pr->Bt(), Cm, n, pr->H(), mb, X0, ldx0, X, ldx, o, iters_out, info,
                       (double*)part, part_doubles);
}
