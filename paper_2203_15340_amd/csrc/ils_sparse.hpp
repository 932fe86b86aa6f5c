// ils_sparse.hpp -- the sparse matrix behind the opaque ils_csr of
// include/ils.h and the launchers of its kernels (k_sparse.hip).
#pragma once
#include "ils_common.hpp"

// A = [A1; A2] in CSR as given by the caller (device arrays, caller-owned),
// plus a column-major copy (CSC, rows ascending within each column) built and
// owned by the library.  Rows [0, p) form A1; a1len[j] is the number of
// entries of column j that lie in A1 (they come first in the column).
struct ils_csr {
  int device = 0;
  int64_t p = 0, q = 0, m = 0, n = 0, nnz = 0;
  const int64_t* rowptr = nullptr;
  const int32_t* colidx = nullptr;
  const double* val = nullptr;
  int64_t* colptr = nullptr;
  int32_t* rowidx = nullptr;
  double* cval = nullptr;
  int32_t* a1len = nullptr;
  int64_t max_col = 0;  // longest column
};

namespace ils {

constexpr int64_t kSparseMaxN = 20480;  // dense n x n Gram accumulators in LDS
constexpr int kBitBadIndex = 4;         // CSR structure or index out of range

// CSC construction
void launch_csr_check(hipStream_t s, const ils_csr& A, int* colcount, int* bits);
void launch_col_scan(hipStream_t s, int64_t n, const int* colcount, int64_t* colptr, int64_t* max_col);
void launch_csc_scatter(hipStream_t s, const ils_csr& A, int* fill, int32_t* rows_tmp, double* vals_tmp);
void launch_csc_sort(hipStream_t s, const ils_csr& A, const int32_t* rows_tmp, const double* vals_tmp);

// solver building blocks on the sparse A
void launch_vec_finite(hipStream_t s, int64_t m, const double* b, int* bits);
void launch_csc_colpass(hipStream_t s, const ils_csr& A, const double* b, double* g, double* cn);
void launch_csr_residual(hipStream_t s, const ils_csr& A, const double* b, const double* x, double* t,
                         double* r, const int* done);
// Dense G = A_part^T A_part for A1 (second == 0) or A2 (second == 1).
void launch_sparse_gram(hipStream_t s, const ils_csr& A, int second, double* G, int64_t ldg);
void launch_rk_inner_csc(hipStream_t st, const ils_csr& A, const double* tgt, const double* cn, const int* j1,
                         const int* j2, int64_t count, double* w, double* s, double* z, const int* inner_done,
                         const int* outer_done);
void launch_rk_check_csc(hipStream_t st, const ils_csr& A, const double* w, const double* s, double* v,
                         const double* tgt, double* res2, double itol2, const double* tn2, int* inner_done,
                         unsigned* arrive, const int* skip);

}  // namespace ils
