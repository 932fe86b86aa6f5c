/* sparse_oracle.c -- plain reference of the column-major copy of a CSR
 * matrix used by the sparse path.
 *
 * TEST INFRASTRUCTURE ONLY (see ils_oracle.h).  Shares no code with the GPU
 * library.
 *
 * Definition: column j of the CSC holds the entries (i, j, v) of the CSR,
 * ordered by row i, and entries of one (i, j) pair (duplicates) by the bit
 * pattern of v read as an unsigned 64-bit integer.  a1len[j] counts the
 * entries of column j with i < p (the rows of A1).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "ils_oracle.h"

typedef struct {
  int32_t row;
  uint64_t bits;
} entry;

static int cmp_entry(const void* a, const void* b) {
  const entry* x = (const entry*)a;
  const entry* y = (const entry*)b;
  if (x->row != y->row) return x->row < y->row ? -1 : 1;
  if (x->bits != y->bits) return x->bits < y->bits ? -1 : 1;
  return 0;
}

void ora_csr_to_csc(int64_t m, int64_t n, int64_t p, const int64_t* rowptr, const int32_t* colidx,
                    const double* val, int64_t* colptr, int32_t* rowidx, double* cval, int32_t* a1len) {
  int64_t nnz = rowptr[m];
  int64_t* fill = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  entry* tmp = (entry*)malloc(sizeof(entry) * (size_t)(nnz > 0 ? nnz : 1));
  for (int64_t j = 0; j <= n; ++j) colptr[j] = 0;
  for (int64_t e = 0; e < nnz; ++e) colptr[colidx[e] + 1] += 1;
  for (int64_t j = 0; j < n; ++j) colptr[j + 1] += colptr[j];
  for (int64_t i = 0; i < m; ++i)
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int32_t j = colidx[e];
      entry* t = &tmp[colptr[j] + fill[j]++];
      t->row = (int32_t)i;
      memcpy(&t->bits, &val[e], sizeof(double));
    }
  for (int64_t j = 0; j < n; ++j) {
    const int64_t b = colptr[j], L = colptr[j + 1] - b;
    qsort(tmp + b, (size_t)L, sizeof(entry), cmp_entry);
    int32_t c = 0;
    for (int64_t e = b; e < b + L; ++e) {
      rowidx[e] = tmp[e].row;
      memcpy(&cval[e], &tmp[e].bits, sizeof(double));
      c += tmp[e].row < p;
    }
    a1len[j] = c;
  }
  free(tmp);
  free(fill);
}
