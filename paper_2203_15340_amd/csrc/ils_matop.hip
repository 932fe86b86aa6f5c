// ils_matop.hip -- the solver drivers' view of A: each building block
// dispatches to the dense kernels (column-major A) or to the sparse ones
// (CSR + CSC), so SP, SP-RK-RGS and SP-SCD share one driver each.
#include <algorithm>

#include "ils_common.hpp"
#include "ils_runtime.hpp"
#include "ils_sparse.hpp"
#include "k_rand.hpp"

namespace ils {

int check_op(const MatOp& M, const double* b, const double* x, const ils_opts* o) {
  if (!M.sp) return check_problem(M.p, M.q, M.n, M.A, M.lda, b, x, o);
  int st = check_problem(M.p, M.q, M.n, M.sp->val, M.p + M.q, b, x, o);
  if (st != ILS_OK) return st;
  if (o->precision != ILS_PREC_FP64) return ILS_ERR_ARG;  // the sparse Gram products are FP64 only
  return ILS_OK;
}

size_t mat_gram_partials(const MatOp& M) {
  if (M.sp) return 1;
  return std::max({gram_partials_size(M.n, M.p), gram_partials_size(M.n, M.q), gram2_partials_size(M.n, M.p, M.q)});
}

void mat_colpass(hipStream_t s, const MatOp& M, const double* b, double* g, double* cn, int* bits) {
  if (!M.sp) {
    launch_colpass(s, M.p, M.q, M.n, M.A, M.lda, b, g, cn, bits);
    return;
  }
  launch_vec_finite(s, M.p + M.q, b, bits);
  launch_csc_colpass(s, *M.sp, b, g, cn);
}

void mat_residual(hipStream_t s, const MatOp& M, const double* b, const double* x, double* t, double* r,
                  const int* done, const SpStopCheck* chk) {
  if (!M.sp)
    launch_residual(s, M.p, M.q, M.n, M.A, M.lda, b, x, t, r, done, chk);
  else
    launch_csr_residual(s, *M.sp, b, x, t, r, done);
}

void mat_gram(hipStream_t s, const MatOp& M, int second, int precision, void* part, double* G, int64_t ldg,
              hipEvent_t mid) {
  if (M.sp) {
    launch_sparse_gram(s, *M.sp, second, G, ldg);
    if (mid) (void)hipEventRecord(mid, s);
    return;
  }
  if (second)
    launch_gram_f64(s, M.q, M.n, M.A + M.p, M.lda, (double*)part, G, ldg, mid);
  else if (precision == ILS_PREC_MIXED)
    launch_gram_f32(s, M.p, M.n, M.A, M.lda, (float*)part, G, ldg, mid);
  else
    launch_gram_f64(s, M.p, M.n, M.A, M.lda, (double*)part, G, ldg, mid);
}

void mat_rk_inner(hipStream_t st, const MatOp& M, const double* tgt, const double* cn, const int* j1,
                  const int* j2, int64_t count, double* w, double* s, double* z, const int* inner_done,
                  const int* outer_done) {
  if (M.sp)
    launch_rk_inner_csc(st, *M.sp, tgt, cn, j1, j2, count, w, s, z, inner_done, outer_done);
  else
    launch_rk_inner(st, M.A, M.lda, M.p, tgt, cn, j1, j2, count, w, s, z, inner_done, outer_done);
}

void mat_rk_check(hipStream_t st, const MatOp& M, const double* w, const double* s, double* v, const double* tgt,
                  double* res2, double itol2, const double* tn2, int* inner_done, unsigned* arrive,
                  const int* skip) {
  if (M.sp)
    launch_rk_check_csc(st, *M.sp, w, s, v, tgt, res2, itol2, tn2, inner_done, arrive, skip);
  else
    launch_rk_check(st, M.A, M.lda, M.p, M.n, w, s, v, tgt, res2, itol2, tn2, inner_done, arrive, skip);
}

}  // namespace ils
