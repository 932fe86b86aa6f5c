// ils_rkmulti_api.hip -- SP-RK-RGS (Algorithm 2) for many right-hand sides
// that share A and one index stream.
//
// Outer step k (per right-hand side r, all in step): stop test at x_k (Sec. 5)
// retires converged columns; the inner target is A2^T A2 x_k + A^T J b_r
// (paper form) or the residual A^T J (b_r - A x_k) (correction form); the
// inner steps run in blocks shared by every column (k_rkmulti.hip) on the
// draws of ils_rk_solve with the same seed, so each column follows the
// iterates it would follow alone; x_{k+1} = z (paper) or x_k + z.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ils_common.hpp"
#include "ils_runtime.hpp"
#include "k_rand.hpp"

using namespace ils;

#define HIPCHK(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return ILS_ERR_HIP; \
  } while (0)

namespace {

int fail_rkm(ils_info* info, int st) {
  if (info) {
    memset(info, 0, sizeof(*info));
    info->status = st;
    info->rr = NAN;
    info->rel_err = -1.0;
  }
  return st;
}

// frozen[r] = column retired, or its inner target is zero (nothing to solve)
__global__ void k_rkm_freeze0(int64_t N, const int* __restrict__ active, const double* __restrict__ tn2,
                              double itol2, int check, int* __restrict__ frozen) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  frozen[r] = !active[r] || (check && tn2[r] <= itol2 * tn2[r]);
}

// x_{k+1} = z (paper form) or x_k + z (correction form) for live columns;
// retired columns keep x_k.  A non-finite entry raises the flag.
__global__ void k_rkm_update(int64_t n, int64_t N, const double* __restrict__ Xk, const double* __restrict__ Z,
                             int correction, const int* __restrict__ active, double* __restrict__ Xn, int* bits) {
  const int64_t total = n * N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t r = e / n;
    double v = Xk[e];
    if (active[r]) v = correction ? v + Z[e] : Z[e];
    if (!isfinite(v)) atomicOr(bits, kBitNonfinite);
    Xn[e] = v;
  }
}

int blocks_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

}  // namespace

extern "C" int ils_rk_solve_multi(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                                  int64_t nrhs, const double* B, int64_t ldb, const double* X0, int64_t ldx0,
                                  double* X, int64_t ldx, const ils_opts* o, int64_t* iters_out,
                                  ils_info* info) {
  if (!h) return fail_rkm(info, ILS_ERR_ARG);
  int st = check_problem(p, q, n, A, lda, B, X, o);
  if (st != ILS_OK) return fail_rkm(info, st);
  const int64_t m = p + q;
  if (nrhs < 1 || nrhs > ((int64_t)1 << 20) || ldb < m || ldx < n || (X0 && ldx0 < n))
    return fail_rkm(info, ILS_ERR_ARG);
  if (o->precision != ILS_PREC_FP64) return fail_rkm(info, ILS_ERR_ARG);
  if (hipSetDevice(h->device) != hipSuccess) return fail_rkm(info, ILS_ERR_HIP);
  hipStream_t s = h->stream;
  const bool paper = o->form == ILS_FORM_PAPER;
  const bool fixed = o->stop_rule == ILS_STOP_FIXED;
  const bool rr = o->stop_rule == ILS_STOP_RR;
  const int64_t max_inner = o->max_inner >= 0 ? o->max_inner : 1000 * n;
  const int64_t check = o->inner_check > 0 ? o->inner_check : n;
  const int64_t chunk = fixed ? 4096 : check;
  const double itol = o->inner_tol > 0.0 ? o->inner_tol : (paper ? 1e-8 : 1e-2);
  const size_t nN = sizeof(double) * (size_t)n * (size_t)nrhs;
  const size_t pN = sizeof(double) * (size_t)p * (size_t)nrhs;
  const size_t fz_bytes = (sizeof(int) * (size_t)nrhs + 7) / 8 * 8;
  double *cn, *prefix, *G, *G2 = nullptr, *Xa, *Xb, *R, *tv, *W, *S, *Z, *T, *V, *tn2, *metric, *den, *g0, *scr;
  int *jj, *act, *frozen;
  int64_t* iters;
  void* part;
  MatOp M;
  M.p = p;
  M.q = q;
  M.n = n;
  M.A = A;
  M.lda = lda;
  if ((st = h->need(kBufCn, sizeof(double) * n, (void**)&cn)) ||
      (st = h->need(kBufPrefix, sizeof(double) * n, (void**)&prefix)) ||
      (st = h->need(kBufG, sizeof(double) * n, (void**)&g0)) ||
      (st = h->need(kBufMG, nN, (void**)&G)) ||
      (paper && (st = h->need(kBufG2, sizeof(double) * n * n, (void**)&G2))) ||
      (st = h->need(kBufMX0, nN, (void**)&Xa)) || (st = h->need(kBufMX1, nN, (void**)&Xb)) ||
      (st = h->need(kBufMR, nN, (void**)&R)) ||
      (st = h->need(kBufT, sizeof(double) * residual_scratch(m, n), (void**)&tv)) ||
      (st = h->need(kBufPart, gram_partials_size(n, q) * sizeof(double), &part)) ||
      (st = h->need(kBufRmW, pN, (void**)&W)) || (st = h->need(kBufRmS, pN, (void**)&S)) ||
      (st = h->need(kBufRmZ, nN, (void**)&Z)) || (st = h->need(kBufRmT, nN, (void**)&T)) ||
      (st = h->need(kBufRmV, sizeof(double) * (size_t)(p + n) * kMR, (void**)&V)) ||
      (st = h->need(kBufRmF, fz_bytes + sizeof(double) * nrhs, (void**)&frozen)) ||
      (st = h->need(kBufMAct, sizeof(int) * nrhs, (void**)&act)) ||
      (st = h->need(kBufMIters, sizeof(int64_t) * nrhs, (void**)&iters)) ||
      (st = h->need(kBufMMetric, sizeof(double) * nrhs, (void**)&metric)) ||
      (st = h->need(kBufMDen, sizeof(double) * nrhs, (void**)&den)) ||
      (st = h->need(kBufIdx, sizeof(int) * 2 * chunk, (void**)&jj)) ||
      (st = h->need(kBufRkb, sizeof(double) * rk_multi_scratch(p), (void**)&scr)))
    return fail_rkm(info, st);
  tn2 = (double*)((char*)frozen + fz_bytes);  // the flags, then the target norms
  double* AtV = V + (size_t)p * kMR;

  LoopState* ds = h->st;
  HIPCHK(hipMemsetAsync(ds, 0, sizeof(LoopState), s));
  if (h->timing()) HIPCHK(hipEventRecord(h->ev0, s));
  // column norms of A1 (the sampling weights) and the screen of A, b_1
  launch_colpass(s, p, q, n, A, lda, B, g0, cn, &ds->bits);
  launch_zero_col_check(s, n, cn, &ds->bits);
  launch_prefix(s, n, cn, 1, prefix);
  // A^T J B (rows p.. of B enter negated)
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
  gb.C = G;
  gb.ldc = n;
  launch_gemm_tn(s, gb);
  if (paper) launch_gram_f64(s, q, n, A + p, lda, (double*)part, G2, n);
  if (rr) launch_colnorm2(s, n, nrhs, G, n, den);
  else if (o->stop_rule == ILS_STOP_XREF) launch_colnorm2(s, n, nrhs, o->x_ref, n, den);
  launch_mat_copy(s, n, nrhs, X0, ldx0, Xa, n);
  launch_fill_int(s, nrhs, 1, act);

  MultiMetricArgs ma = {};
  ma.n = n;
  ma.N = nrhs;
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

  double* cur = Xa;
  double* nxt = Xb;
  int64_t k = 0, inner_total = 0;
  int status = ILS_OK;
  std::vector<int> hfz(nrhs);
  auto residuals = [&](const double* Xk) {
    for (int64_t r = 0; r < nrhs; ++r) mat_residual(s, M, B + r * ldb, Xk + r * n, tv, R + r * n, nullptr);
  };
  for (;; ++k) {
    bool have_r = false;
    if (!fixed) {
      if (rr) {
        residuals(cur);
        have_r = true;
      }
      ma.V = rr ? R : cur;
      HIPCHK(hipMemsetAsync(&ds->nactive, 0, sizeof(int), s));
      launch_multi_metric(s, ma, k);
    }
    if (h->timing()) HIPCHK(hipEventRecord(h->ev1, s));
    if ((st = read_state(h))) return fail_rkm(info, st);
    {
      const LoopState& hs = *h->st_host;
      if (hs.bits & kBitNotSpd) return fail_rkm(info, ILS_ERR_NOT_SPD);
      if (hs.bits & kBitStall) return fail_rkm(info, ILS_ERR_HIP);
      if (hs.bits & kBitNonfinite) {
        if (k == 0) return fail_rkm(info, ILS_ERR_NONFINITE);  // A or b
        status = ILS_ERR_NONFINITE;
        break;
      }
      if (!fixed && hs.nactive == 0) break;
    }
    if (k == o->max_outer) {
      if (!fixed) status = ILS_ERR_NO_CONVERGENCE;
      break;
    }
    // inner targets and their norms
    if (paper) {
      GemmTnArgs gt = {};
      gt.M = n;
      gt.N = nrhs;
      gt.K = n;
      gt.X = G2;
      gt.ldx = n;
      gt.Y = cur;
      gt.ldy = n;
      gt.kneg = n;
      gt.alpha = 1.0;
      gt.beta = 1.0;
      gt.C0 = G;
      gt.ldc0 = n;
      gt.C = T;
      gt.ldc = n;
      launch_gemm_tn(s, gt);
    } else {
      if (!have_r) residuals(cur);
      launch_mat_copy(s, n, nrhs, R, n, T, n);
    }
    launch_colnorm2(s, n, nrhs, T, n, tn2);
    hipLaunchKernelGGL(k_rkm_freeze0, dim3((unsigned)((nrhs + 255) / 256)), dim3(256), 0, s, nrhs, (const int*)act,
                       (const double*)tn2, itol * itol, fixed ? 0 : 1, frozen);
    HIPCHK(hipMemsetAsync(W, 0, pN, s));
    HIPCHK(hipMemsetAsync(S, 0, pN, s));
    HIPCHK(hipMemsetAsync(Z, 0, nN, s));
    int64_t t = 0;
    bool all_frozen = false;
    if (!fixed) {
      HIPCHK(hipMemcpyAsync(hfz.data(), frozen, sizeof(int) * nrhs, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      all_frozen = std::all_of(hfz.begin(), hfz.end(), [](int v) { return v != 0; });
    }
    while (t < max_inner && !all_frozen) {
      const int64_t cnt = std::min(chunk, max_inner - t);
      launch_rk_draw(s, o->seed, (uint64_t)k + o->stream_offset, t, cnt, prefix, n, jj, jj + chunk);
      for (int64_t g0c = 0; g0c < nrhs; g0c += kMR) {
        const int Rg = (int)std::min<int64_t>(kMR, nrhs - g0c);
        launch_rk_multi_blocks(s, A, lda, p, Rg, T + g0c * n, n, cn, jj, jj + chunk, cnt, W + g0c * p,
                               S + g0c * p, p, Z + g0c * n, n, frozen + g0c, scr, &ds->arrive3);
      }
      t += cnt;
      if (!fixed && t % check == 0) {
        for (int64_t g0c = 0; g0c < nrhs; g0c += kMR) {
          const int Rg = (int)std::min<int64_t>(kMR, nrhs - g0c);
          launch_rkm_check(s, A, lda, p, n, Rg, W + g0c * p, S + g0c * p, p, V, AtV, T + g0c * n, n, tn2 + g0c,
                           itol * itol, frozen + g0c);
        }
        HIPCHK(hipMemcpyAsync(hfz.data(), frozen, sizeof(int) * nrhs, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        all_frozen = std::all_of(hfz.begin(), hfz.end(), [](int v) { return v != 0; });
      }
    }
    inner_total += t;
    hipLaunchKernelGGL(k_rkm_update, dim3(blocks_for(n * nrhs)), dim3(256), 0, s, n, nrhs, (const double*)cur,
                       (const double*)Z, paper ? 0 : 1, (const int*)act, nxt, &ds->bits);
    std::swap(cur, nxt);
  }
  launch_mat_copy(s, n, nrhs, cur, n, X, ldx);
  HIPCHK(hipGetLastError());
  std::vector<int> hact(nrhs);
  std::vector<int64_t> hit(nrhs, 0);
  std::vector<double> hmet(nrhs, 0.0);
  HIPCHK(hipMemcpyAsync(hact.data(), act, sizeof(int) * nrhs, hipMemcpyDeviceToHost, s));
  if (!fixed) HIPCHK(hipMemcpyAsync(hit.data(), iters, sizeof(int64_t) * nrhs, hipMemcpyDeviceToHost, s));
  if (rr) HIPCHK(hipMemcpyAsync(hmet.data(), metric, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
  double worst_rel = -1.0;
  if (o->x_ref) {
    MultiMetricArgs mr = ma;
    mr.V = cur;
    mr.stop_rule = ILS_STOP_XREF;
    mr.report = 1;
    if (o->stop_rule != ILS_STOP_XREF) launch_colnorm2(s, n, nrhs, o->x_ref, n, den);
    std::vector<double> rel(nrhs);
    launch_multi_metric(s, mr, k);
    HIPCHK(hipMemcpyAsync(rel.data(), metric, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (double v : rel) worst_rel = std::max(worst_rel, v);
  }
  HIPCHK(hipStreamSynchronize(s));
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
    info->inner_iters = inner_total;
    info->rr = rr ? worst_rr : NAN;
    info->rel_err = worst_rel;
    float ms = 0.0f;
    info->device_ms = (h->timing() && hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) ? ms : 0.0;
  }
  return status;
}
