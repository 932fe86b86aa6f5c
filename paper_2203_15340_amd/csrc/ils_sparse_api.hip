// ils_sparse_api.hip -- sparse A behind include/ils.h: creation of the CSR
// handle (checks, CSC copy with rows ascending per column), the three
// solvers on it, and its component entry points.
#include <math.h>
#include <string.h>

#include "ils_common.hpp"
#include "ils_runtime.hpp"
#include "ils_sparse.hpp"

using namespace ils;

#define HIPCHK(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return ILS_ERR_HIP; \
  } while (0)

static void free_csr(ils_csr* A) {
  if (!A) return;
  void* dev[] = {A->colptr, A->rowidx, A->cval, A->a1len};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  delete A;
}

extern "C" int ils_csr_create(ils_handle* h, int64_t p, int64_t q, int64_t n, int64_t nnz, const int64_t* rowptr,
                              const int32_t* colidx, const double* val, ils_csr** out) {
  if (!h || !out || !rowptr || !colidx || !val) return ILS_ERR_ARG;
  const int64_t m = p + q;
  if (p < 0 || q < 0 || n < 1 || n > kSparseMaxN || m < 1 || m >= ((int64_t)1 << 31) || nnz < 1 ||
      nnz >= ((int64_t)1 << 31))
    return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  hipStream_t s = h->stream;
  ils_csr* A = new ils_csr();
  A->device = h->device;
  A->p = p;
  A->q = q;
  A->m = m;
  A->n = n;
  A->nnz = nnz;
  A->rowptr = rowptr;
  A->colidx = colidx;
  A->val = val;
  int *cnt = nullptr, *fill = nullptr, *bits = nullptr;
  int64_t* maxc = nullptr;
  int32_t* rows_tmp = nullptr;
  double* vals_tmp = nullptr;
  int st = ILS_OK;
  auto cleanup = [&]() {
    void* tmp[] = {cnt, fill, bits, maxc, rows_tmp, vals_tmp};
    for (void* t : tmp)
      if (t) (void)hipFree(t);
  };
  if (hipMalloc((void**)&cnt, sizeof(int) * n) != hipSuccess || hipMalloc((void**)&fill, sizeof(int) * n) != hipSuccess ||
      hipMalloc((void**)&bits, sizeof(int)) != hipSuccess || hipMalloc((void**)&maxc, sizeof(int64_t)) != hipSuccess ||
      hipMalloc((void**)&rows_tmp, sizeof(int32_t) * nnz) != hipSuccess ||
      hipMalloc((void**)&vals_tmp, sizeof(double) * nnz) != hipSuccess ||
      hipMalloc((void**)&A->colptr, sizeof(int64_t) * (n + 1)) != hipSuccess ||
      hipMalloc((void**)&A->rowidx, sizeof(int32_t) * nnz) != hipSuccess ||
      hipMalloc((void**)&A->cval, sizeof(double) * nnz) != hipSuccess ||
      hipMalloc((void**)&A->a1len, sizeof(int32_t) * n) != hipSuccess) {
    cleanup();
    free_csr(A);
    return ILS_ERR_ALLOC;
  }
  int hbits = 0;
  if (hipMemsetAsync(cnt, 0, sizeof(int) * n, s) != hipSuccess || hipMemsetAsync(fill, 0, sizeof(int) * n, s) != hipSuccess ||
      hipMemsetAsync(bits, 0, sizeof(int), s) != hipSuccess) {
    st = ILS_ERR_HIP;
  } else {
    launch_csr_check(s, *A, cnt, bits);
    if (hipMemcpyAsync(&hbits, bits, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = ILS_ERR_HIP;
    else if (hbits & kBitBadIndex)
      st = ILS_ERR_ARG;
    else if (hbits & kBitNonfinite)
      st = ILS_ERR_NONFINITE;
  }
  if (st == ILS_OK) {
    // the structure is valid: every scatter position below lies in [0, nnz)
    launch_col_scan(s, n, cnt, A->colptr, maxc);
    launch_csc_scatter(s, *A, fill, rows_tmp, vals_tmp);
    launch_csc_sort(s, *A, rows_tmp, vals_tmp);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&A->max_col, maxc, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = ILS_ERR_HIP;
  }
  cleanup();
  if (st != ILS_OK) {
    free_csr(A);
    return st;
  }
  *out = A;
  return ILS_OK;
}

extern "C" int ils_csr_destroy(ils_csr* A) {
  if (!A) return ILS_ERR_ARG;
  (void)hipSetDevice(A->device);
  free_csr(A);
  return ILS_OK;
}

extern "C" int ils_csr_export_csc(const ils_csr* A, int64_t* colptr, int32_t* rowidx, double* val,
                                  int32_t* a1len) {
  if (!A || !colptr || !rowidx || !val || !a1len) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(A->device));
  HIPCHK(hipMemcpy(colptr, A->colptr, sizeof(int64_t) * (A->n + 1), hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(rowidx, A->rowidx, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(val, A->cval, sizeof(double) * A->nnz, hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(a1len, A->a1len, sizeof(int32_t) * A->n, hipMemcpyDeviceToDevice));
  return ILS_OK;
}

static int csr_op(ils_handle* h, const ils_csr* A, MatOp& M) {
  if (!h || !A || A->device != h->device) return ILS_ERR_ARG;
  M.p = A->p;
  M.q = A->q;
  M.n = A->n;
  M.sp = A;
  return ILS_OK;
}

static int fail_csr(ils_info* info, int st) {
  if (info) {
    memset(info, 0, sizeof(*info));
    info->status = st;
    info->rr = NAN;
    info->rel_err = -1.0;
  }
  return st;
}

extern "C" int ils_sp_solve_csr(ils_handle* h, const ils_csr* A, const double* b, const double* x0, double* x,
                                const ils_opts* o, ils_info* info) {
  MatOp M;
  const int st = csr_op(h, A, M);
  return st ? fail_csr(info, st) : sp_solve_op(h, M, b, x0, x, o, info);
}

extern "C" int ils_rk_solve_csr(ils_handle* h, const ils_csr* A, const double* b, const double* x0, double* x,
                                const ils_opts* o, ils_info* info) {
  MatOp M;
  const int st = csr_op(h, A, M);
  return st ? fail_csr(info, st) : rk_solve_op(h, M, b, x0, x, o, info);
}

extern "C" int ils_rgs_solve_csr(ils_handle* h, const ils_csr* A, const double* b, const double* x0, double* x,
                                 const ils_opts* o, ils_info* info) {
  MatOp M;
  const int st = csr_op(h, A, M);
  return st ? fail_csr(info, st) : rgs_solve_op(h, M, b, x0, x, o, info);
}

extern "C" int ils_csr_gram(ils_handle* h, const ils_csr* A, int32_t part, double* G, int64_t ldg) {
  MatOp M;
  int st = csr_op(h, A, M);
  if (st) return st;
  if (!G || ldg < A->n || (part != 0 && part != 1)) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  mat_gram(h->stream, M, part, ILS_PREC_FP64, nullptr, G, ldg);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return ILS_OK;
}

extern "C" int ils_csr_colpass(ils_handle* h, const ils_csr* A, const double* b, double* g, double* colnorm2) {
  MatOp M;
  int st = csr_op(h, A, M);
  if (st) return st;
  if (!b || !g) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  HIPCHK(hipMemsetAsync(h->st, 0, sizeof(LoopState), h->stream));
  mat_colpass(h->stream, M, b, g, colnorm2, &h->st->bits);
  HIPCHK(hipGetLastError());
  if ((st = read_state(h))) return st;
  return (h->st_host->bits & kBitNonfinite) ? ILS_ERR_NONFINITE : ILS_OK;
}

extern "C" int ils_csr_residual(ils_handle* h, const ils_csr* A, const double* b, const double* x, double* r) {
  MatOp M;
  int st = csr_op(h, A, M);
  if (st) return st;
  if (!b || !x || !r) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  double* tv;
  if ((st = h->need(kBufT, sizeof(double) * A->m, (void**)&tv))) return st;
  mat_residual(h->stream, M, b, x, tv, r, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return ILS_OK;
}
