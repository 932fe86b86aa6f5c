// k_sparse.hip -- kernels of the sparse (CSR) path: building the CSC copy,
// the column pass (A^T J b and column norms of A1, Alg. 1 step 4 and the
// sampling weights of Alg. 2), the residual A^T J (b - A x) (eq. Sec12), the
// dense Gram matrices A1^T A1 and A2^T A2 from the sparse factors (Alg. 1
// steps 2-3), and the SP-RK-RGS inner steps on sparse columns of A1
// (Alg. 2 steps 8-11).
#include "ils_common.hpp"
#include "ils_sparse.hpp"

namespace ils {

// ------------------------------------------------------------------ CSC build
__global__ __launch_bounds__(256) void k_csr_check(int64_t m, int64_t n, int64_t nnz,
                                                   const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ colidx,
                                                   const double* __restrict__ val, int* __restrict__ colcount,
                                                   int* bits) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x, stride = (int64_t)gridDim.x * 256;
  if (gid == 0 && (rowptr[0] != 0 || rowptr[m] != nnz)) atomicOr(bits, kBitBadIndex);
  for (int64_t i = gid; i < m; i += stride) {
    const int64_t r0 = rowptr[i], r1 = rowptr[i + 1];
    if (r0 < 0 || r1 < r0 || r1 > nnz) {
      atomicOr(bits, kBitBadIndex);
      continue;
    }
    for (int64_t e = r0; e < r1; ++e) {
      const int c = colidx[e];
      if (c < 0 || c >= n) {
        atomicOr(bits, kBitBadIndex);
        continue;
      }
      if (!isfinite(val[e])) atomicOr(bits, kBitNonfinite);
      atomicAdd(&colcount[c], 1);
    }
  }
}

void launch_csr_check(hipStream_t s, const ils_csr& A, int* colcount, int* bits) {
  int64_t blocks = (A.m + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_csr_check, dim3((unsigned)blocks), dim3(256), 0, s, A.m, A.n, A.nnz, A.rowptr, A.colidx,
                     A.val, colcount, bits);
}

// Exclusive scan of the column counts (one workgroup) and the longest column.
__global__ __launch_bounds__(1024) void k_col_scan(int64_t n, const int* __restrict__ cnt,
                                                   int64_t* __restrict__ colptr, int64_t* __restrict__ maxc) {
  __shared__ int64_t buf[1024];
  __shared__ int64_t red[16];
  const int tid = threadIdx.x;
  int64_t carry = 0, lmax = 0;
  for (int64_t base = 0; base < n; base += 1024) {
    const int64_t v = base + tid < n ? cnt[base + tid] : 0;
    lmax = v > lmax ? v : lmax;
    buf[tid] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int64_t a = tid >= off ? buf[tid - off] : 0;
      __syncthreads();
      buf[tid] += a;
      __syncthreads();
    }
    if (base + tid < n) colptr[base + tid] = carry + buf[tid] - v;
    carry += buf[1023];
    __syncthreads();
  }
  if (tid == 0) colptr[n] = carry;
  // maximum over the block
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int64_t o = __shfl_xor(lmax, off, kWave);
    lmax = o > lmax ? o : lmax;
  }
  if ((tid & 63) == 0) red[tid >> 6] = lmax;
  __syncthreads();
  if (tid == 0) {
    int64_t mx = 0;
    for (int i = 0; i < 16; ++i) mx = red[i] > mx ? red[i] : mx;
    *maxc = mx;
  }
}

void launch_col_scan(hipStream_t s, int64_t n, const int* colcount, int64_t* colptr, int64_t* max_col) {
  hipLaunchKernelGGL(k_col_scan, dim3(1), dim3(1024), 0, s, n, colcount, colptr, max_col);
}

__global__ __launch_bounds__(256) void k_csc_scatter(int64_t m, const int64_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ colidx,
                                                     const double* __restrict__ val,
                                                     const int64_t* __restrict__ colptr, int* __restrict__ fill,
                                                     int32_t* __restrict__ rows_tmp, double* __restrict__ vals_tmp) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int c = colidx[e];
      const int64_t pos = colptr[c] + atomicAdd(&fill[c], 1);
      rows_tmp[pos] = (int32_t)i;
      vals_tmp[pos] = val[e];
    }
  }
}

void launch_csc_scatter(hipStream_t s, const ils_csr& A, int* fill, int32_t* rows_tmp, double* vals_tmp) {
  int64_t blocks = (A.m + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_csc_scatter, dim3((unsigned)blocks), dim3(256), 0, s, A.m, A.rowptr, A.colidx, A.val,
                     (const int64_t*)A.colptr, fill, rows_tmp, vals_tmp);
}

// Order of entries within a column: by row, then by the value's bit pattern
// (only duplicates of one (row, column) pair tie on the row), so the result
// does not depend on the order the scatter's atomics happened to take.
__device__ inline bool key_less(int ra, uint64_t va, int rb, uint64_t vb) {
  return ra < rb || (ra == rb && va < vb);
}

constexpr int kSortLds = 4096;

// One workgroup per column: sort the column's entries, write them to the
// final CSC arrays and count the entries with row < p (the A1 part).
__global__ __launch_bounds__(256) void k_csc_sort(int64_t p, const int64_t* __restrict__ colptr,
                                                  const int32_t* __restrict__ rows_tmp,
                                                  const double* __restrict__ vals_tmp, int32_t* __restrict__ rowidx,
                                                  double* __restrict__ cval, int32_t* __restrict__ a1len) {
  __shared__ int kr[kSortLds];
  __shared__ uint64_t kv[kSortLds];
  __shared__ int red[4];
  const int64_t c = blockIdx.x;
  const int64_t base = colptr[c], L = colptr[c + 1] - base;
  const int tid = threadIdx.x;
  int cnt = 0;
  if (L <= kSortLds) {
    int P = 1;
    while (P < L) P <<= 1;
    for (int e = tid; e < P; e += 256) {
      kr[e] = e < L ? rows_tmp[base + e] : 0x7FFFFFFF;
      kv[e] = e < L ? (uint64_t)__double_as_longlong(vals_tmp[base + e]) : ~0ull;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = tid; i < P; i += 256) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const bool up = (i & k) == 0;
            const bool sw = up ? key_less(kr[ixj], kv[ixj], kr[i], kv[i]) : key_less(kr[i], kv[i], kr[ixj], kv[ixj]);
            if (sw) {
              const int tr = kr[i];
              kr[i] = kr[ixj];
              kr[ixj] = tr;
              const uint64_t tv = kv[i];
              kv[i] = kv[ixj];
              kv[ixj] = tv;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int64_t e = tid; e < L; e += 256) {
      rowidx[base + e] = kr[e];
      cval[base + e] = __longlong_as_double((long long)kv[e]);
      cnt += kr[e] < p;
    }
  } else {
    // long column: rank of every entry among the column's keys
    for (int64_t e = tid; e < L; e += 256) {
      const int re = rows_tmp[base + e];
      const uint64_t ve = (uint64_t)__double_as_longlong(vals_tmp[base + e]);
      int64_t rank = 0;
      for (int64_t f = 0; f < L; ++f) {
        const int rf = rows_tmp[base + f];
        const uint64_t vf = (uint64_t)__double_as_longlong(vals_tmp[base + f]);
        rank += key_less(rf, vf, re, ve) || (rf == re && vf == ve && f < e);
      }
      rowidx[base + rank] = re;
      cval[base + rank] = __longlong_as_double((long long)ve);
      cnt += re < p;
    }
  }
  // A1 part length
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
  if ((tid & 63) == 0) red[tid >> 6] = cnt;
  __syncthreads();
  if (tid == 0) a1len[c] = red[0] + red[1] + red[2] + red[3];
}

void launch_csc_sort(hipStream_t s, const ils_csr& A, const int32_t* rows_tmp, const double* vals_tmp) {
  hipLaunchKernelGGL(k_csc_sort, dim3((unsigned)A.n), dim3(256), 0, s, A.p, (const int64_t*)A.colptr, rows_tmp,
                     vals_tmp, A.rowidx, A.cval, A.a1len);
}

// ------------------------------------------------------------------ vectors
__global__ void k_vec_finite(int64_t m, const double* __restrict__ b, int* bits) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
    bad |= !isfinite(b[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(bits, kBitNonfinite);
}

void launch_vec_finite(hipStream_t s, int64_t m, const double* b, int* bits) {
  int64_t blocks = (m + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_vec_finite, dim3((unsigned)blocks), dim3(256), 0, s, m, b, bits);
}

// One wavefront per column: g_j = A1_(j)^T b1 - A2_(j)^T b2, cn_j = ||A1_(j)||^2.
__global__ __launch_bounds__(256) void k_csc_colpass(int64_t n, const int64_t* __restrict__ colptr,
                                                     const int32_t* __restrict__ rowidx,
                                                     const double* __restrict__ cval,
                                                     const int32_t* __restrict__ a1len,
                                                     const double* __restrict__ b, double* __restrict__ g,
                                                     double* __restrict__ cn) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= n) return;
  const int64_t base = colptr[c], L = colptr[c + 1] - base, l1 = a1len[c];
  double sg = 0.0, sc = 0.0;
  for (int64_t e = lane; e < L; e += 64) {
    const double v = cval[base + e];
    const double bv = b[rowidx[base + e]];
    if (e < l1) {
      sg += v * bv;
      sc += v * v;
    } else {
      sg -= v * bv;
    }
  }
  sg = wave_sum(sg);
  sc = wave_sum(sc);
  if (lane == 0) {
    g[c] = sg;
    if (cn) cn[c] = sc;
  }
}

void launch_csc_colpass(hipStream_t s, const ils_csr& A, const double* b, double* g, double* cn) {
  hipLaunchKernelGGL(k_csc_colpass, dim3((unsigned)((A.n + 3) / 4)), dim3(256), 0, s, A.n,
                     (const int64_t*)A.colptr, (const int32_t*)A.rowidx, (const double*)A.cval,
                     (const int32_t*)A.a1len, b, g, cn);
}

// t = J (b - A x): 16 lanes per row of the CSR.
__global__ __launch_bounds__(256) void k_csr_resid(int64_t m, int64_t p, const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ colidx,
                                                   const double* __restrict__ val, const double* __restrict__ b,
                                                   const double* __restrict__ x, double* __restrict__ t,
                                                   const int* done) {
  if (done && *(volatile const int*)done) return;
  const int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4;
  const int sub = threadIdx.x & 15;
  double a = 0.0;
  if (row < m)
    for (int64_t e = rowptr[row] + sub; e < rowptr[row + 1]; e += 16) a += val[e] * x[colidx[e]];
  a = row16_sum(a);
  if (row < m && sub == 0) {
    const double d = b[row] - a;
    t[row] = row < p ? d : -d;
  }
}

// r = A^T t: one wavefront per column.
__global__ __launch_bounds__(256) void k_csc_atv(int64_t n, const int64_t* __restrict__ colptr,
                                                 const int32_t* __restrict__ rowidx, const double* __restrict__ cval,
                                                 const double* __restrict__ t, double* __restrict__ r,
                                                 const int* done) {
  if (done && *(volatile const int*)done) return;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= n) return;
  const int64_t base = colptr[c], L = colptr[c + 1] - base;
  double a = 0.0;
  for (int64_t e = lane; e < L; e += 64) a += cval[base + e] * t[rowidx[base + e]];
  a = wave_sum(a);
  if (lane == 0) r[c] = a;
}

void launch_csr_residual(hipStream_t s, const ils_csr& A, const double* b, const double* x, double* t, double* r,
                         const int* done) {
  const int64_t blocks = (A.m * 16 + 255) / 256;
  hipLaunchKernelGGL(k_csr_resid, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, A.m, A.p, A.rowptr,
                     A.colidx, A.val, b, x, t, done);
  hipLaunchKernelGGL(k_csc_atv, dim3((unsigned)((A.n + 3) / 4)), dim3(256), 0, s, A.n, (const int64_t*)A.colptr,
                     (const int32_t*)A.rowidx, (const double*)A.cval, (const double*)t, r, done);
}

// ------------------------------------------------------------------ Gram
// One workgroup per column j of G = A_part^T A_part (lower triangle k >= j,
// mirrored): for every entry a_ij of column j in the part, add a_ij * a_ik
// for the entries a_ik (k >= j) of CSR row i into an LDS accumulator of
// length n.  Each wavefront owns a private accumulator and takes 64 entries
// of the column at a time, one CSR row per lane (LDS atomics; lanes that hit
// the same k in one instruction are applied by the LDS in a fixed order);
// the copies are added in a fixed order.
__global__ void k_sparse_gram(int64_t n, int second, const int64_t* __restrict__ rowptr,
                              const int32_t* __restrict__ colidx, const double* __restrict__ val,
                              const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                              const double* __restrict__ cval, const int32_t* __restrict__ a1len,
                              double* __restrict__ G, int64_t ldg) {
  extern __shared__ double acc[];
  const int copies = blockDim.x >> 6;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t j = blockIdx.x;
  for (int64_t k = threadIdx.x; k < (int64_t)copies * n; k += blockDim.x) acc[k] = 0.0;
  __syncthreads();
  const int64_t base = colptr[j], L = colptr[j + 1] - base, l1 = a1len[j];
  const int64_t e0 = second ? l1 : 0, e1 = second ? L : l1;
  double* my = acc + (int64_t)w * n;
  // lane l of wave w walks CSR row i of column entry e = e0 + 64 (w + copies t) + l;
  // the 64 rows of one step load their index ranges together
  for (int64_t e = e0 + (int64_t)w * 64 + lane; e - lane < e1; e += (int64_t)copies * 64) {
    const bool live = e < e1;
    const int64_t i = live ? rowidx[base + e] : 0;
    const double a = live ? cval[base + e] : 0.0;
    const int64_t f0 = live ? rowptr[i] : 0, f1 = live ? rowptr[i + 1] : 0;
    for (int64_t f = f0; f < f1; ++f) {
      const int k = colidx[f];
      if (k >= j) atomicAdd(&my[k], a * val[f]);
    }
  }
  __syncthreads();
  for (int64_t k = j + threadIdx.x; k < n; k += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < copies; ++c) s += acc[(int64_t)c * n + k];
    G[k + j * ldg] = s;
    G[j + k * ldg] = s;
  }
}

void launch_sparse_gram(hipStream_t s, const ils_csr& A, int second, double* G, int64_t ldg) {
  static int64_t lds_max = -1;
  if (lds_max < 0)  // the CDNA4 LDS holds 160 KB; allow the kernel all of it
    lds_max = hipFuncSetAttribute((const void*)k_sparse_gram, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024) == hipSuccess ? 160 * 1024 : 64 * 1024;
  int copies = 4;
  while (copies > 1 && (int64_t)copies * A.n * 8 > lds_max) copies >>= 1;
  const size_t lds = (size_t)copies * A.n * sizeof(double);
  hipLaunchKernelGGL(k_sparse_gram, dim3((unsigned)A.n), dim3(64 * copies), lds, s, A.n, second, A.rowptr,
                     A.colidx, A.val, (const int64_t*)A.colptr, (const int32_t*)A.rowidx, (const double*)A.cval,
                     (const int32_t*)A.a1len, G, ldg);
}

// ------------------------------------------------------------------ SP-RK-RGS on sparse columns
// The incremental inner step of Alg. 2 (s = w - A1 z) with the A1 part of
// columns j1, j2 read from the CSC copy.  Rows of the two columns overlap in
// general, so the s update of the Kaczmarz half is made visible to the whole
// workgroup (barrier) before the Gauss-Seidel half reads it.  The column
// draws do not depend on the iterate, so the next step's column data (its
// indices, offsets, lengths, targets, norms, and the row indices and values
// of both columns) are loaded during the current step; a step then waits only
// on its gathers of w and s and its two block sums.  Columns longer than
// kRkSpQ entries per thread take the loop form.
constexpr int kRkSpThreads = 1024;
constexpr int kRkSpQ = 2;

struct RkSpMeta {
  int j1, j2;
  int64_t b1, l1, b2, l2;
  double tg, c1, c2;
};

__global__ __launch_bounds__(kRkSpThreads) void k_rk_inner_csc(
    const int64_t* __restrict__ colptr, const int32_t* __restrict__ rowidx, const double* __restrict__ cval,
    const int32_t* __restrict__ a1len, const double* __restrict__ tgt, const double* __restrict__ cn,
    const int* __restrict__ j1s, const int* __restrict__ j2s, int64_t count, double* __restrict__ w,
    double* __restrict__ s, double* __restrict__ z, const int* inner_done, const int* outer_done) {
  if (*(volatile const int*)inner_done || *(volatile const int*)outer_done) return;
  __shared__ double red[2][kRkSpThreads / kWave];
  const int tid = threadIdx.x;
  auto meta_of = [&](int64_t t) {
    RkSpMeta m;
    m.j1 = j1s[t];
    m.j2 = j2s[t];
    m.b1 = colptr[m.j1];
    m.l1 = a1len[m.j1];
    m.b2 = colptr[m.j2];
    m.l2 = a1len[m.j2];
    m.tg = tgt[m.j1];
    m.c1 = cn[m.j1];
    m.c2 = cn[m.j2];
    return m;
  };
  auto fits = [&](const RkSpMeta& m) { return m.l1 <= kRkSpQ * kRkSpThreads && m.l2 <= kRkSpQ * kRkSpThreads; };
  // this thread's entries e = tid + q T of both columns (row -1: none)
  int32_t r1[kRkSpQ], r2[kRkSpQ], n1[kRkSpQ], n2[kRkSpQ];
  double v1[kRkSpQ], v2[kRkSpQ], u1[kRkSpQ], u2[kRkSpQ];
  auto cols_of = [&](const RkSpMeta& m, int32_t (&ra)[kRkSpQ], double (&va)[kRkSpQ], int32_t (&rb)[kRkSpQ],
                     double (&vb)[kRkSpQ]) {
#pragma unroll
    for (int q = 0; q < kRkSpQ; ++q) {
      const int64_t e = tid + (int64_t)q * kRkSpThreads;
      const bool in1 = e < m.l1, in2 = e < m.l2;
      ra[q] = in1 ? rowidx[m.b1 + e] : -1;
      va[q] = in1 ? cval[m.b1 + e] : 0.0;
      rb[q] = in2 ? rowidx[m.b2 + e] : -1;
      vb[q] = in2 ? cval[m.b2 + e] : 0.0;
    }
  };
  if (count <= 0) return;
#pragma unroll
  for (int q = 0; q < kRkSpQ; ++q) {
    n1[q] = n2[q] = -1;
    u1[q] = u2[q] = 0.0;
  }
  RkSpMeta m = meta_of(0);
  if (fits(m)) cols_of(m, r1, v1, r2, v2);
  for (int64_t t = 0; t < count; ++t) {
    const bool has_next = t + 1 < count;
    RkSpMeta mn = m;
    if (has_next) mn = meta_of(t + 1);
    if (fits(m)) {
      double wv[kRkSpQ], sv[kRkSpQ];
#pragma unroll
      for (int q = 0; q < kRkSpQ; ++q) {
        wv[q] = r1[q] >= 0 ? w[r1[q]] : 0.0;
        sv[q] = r1[q] >= 0 ? s[r1[q]] : 0.0;
      }
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < kRkSpQ; ++q)
        if (r1[q] >= 0) d += v1[q] * wv[q];
      d = block_sum<kRkSpThreads>(d, red[0]);
      const double gam = (m.tg - d) / m.c1;
#pragma unroll
      for (int q = 0; q < kRkSpQ; ++q)
        if (r1[q] >= 0) {
          w[r1[q]] = wv[q] + gam * v1[q];
          s[r1[q]] = sv[q] + gam * v1[q];
        }
      // the next step's columns go out while this one finishes
      if (has_next && fits(mn)) cols_of(mn, n1, u1, n2, u2);
      __syncthreads();
      double s2[kRkSpQ];
#pragma unroll
      for (int q = 0; q < kRkSpQ; ++q) s2[q] = r2[q] >= 0 ? s[r2[q]] : 0.0;
      double d2 = 0.0;
#pragma unroll
      for (int q = 0; q < kRkSpQ; ++q)
        if (r2[q] >= 0) d2 += v2[q] * s2[q];
      d2 = block_sum<kRkSpThreads>(d2, red[1]);
      const double del = d2 / m.c2;
      if (tid == 0) z[m.j2] += del;
#pragma unroll
      for (int q = 0; q < kRkSpQ; ++q)
        if (r2[q] >= 0) s[r2[q]] = s2[q] - del * v2[q];
      __syncthreads();
    } else {
      double d = 0.0;
      for (int64_t e = tid; e < m.l1; e += kRkSpThreads) d += cval[m.b1 + e] * w[rowidx[m.b1 + e]];
      d = block_sum<kRkSpThreads>(d, red[0]);
      const double gam = (m.tg - d) / m.c1;
      for (int64_t e = tid; e < m.l1; e += kRkSpThreads) {
        const int64_t r = rowidx[m.b1 + e];
        const double av = cval[m.b1 + e];
        w[r] += gam * av;
        s[r] += gam * av;
      }
      __syncthreads();
      double d2 = 0.0;
      for (int64_t e = tid; e < m.l2; e += kRkSpThreads) d2 += cval[m.b2 + e] * s[rowidx[m.b2 + e]];
      d2 = block_sum<kRkSpThreads>(d2, red[1]);
      const double del = d2 / m.c2;
      if (tid == 0) z[m.j2] += del;
      for (int64_t e = tid; e < m.l2; e += kRkSpThreads) s[rowidx[m.b2 + e]] -= del * cval[m.b2 + e];
      __syncthreads();
      if (has_next && fits(mn)) cols_of(mn, n1, u1, n2, u2);
    }
    m = mn;
#pragma unroll
    for (int q = 0; q < kRkSpQ; ++q) {
      r1[q] = n1[q];
      v1[q] = u1[q];
      r2[q] = n2[q];
      v2[q] = u2[q];
    }
  }
}

void launch_rk_inner_csc(hipStream_t st, const ils_csr& A, const double* tgt, const double* cn, const int* j1,
                         const int* j2, int64_t count, double* w, double* s, double* z, const int* inner_done,
                         const int* outer_done) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_rk_inner_csc, dim3(1), dim3(kRkSpThreads), 0, st, (const int64_t*)A.colptr,
                     (const int32_t*)A.rowidx, (const double*)A.cval, (const int32_t*)A.a1len, tgt, cn, j1, j2,
                     count, w, s, z, inner_done, outer_done);
}

__global__ void k_sub_vec_sp(int64_t p, const double* __restrict__ w, const double* __restrict__ s,
                             double* __restrict__ v, const int* skip) {
  if (*(volatile const int*)skip) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = w[i] - s[i];
}

// Inner stop test: ||bhat - A1^T (w - s)|| <= tol ||bhat||, one workgroup
// per column; the last workgroup adds the squared entries in column order.
__global__ __launch_bounds__(256) void k_rk_check_csc(int64_t n, const int64_t* __restrict__ colptr,
                                                      const int32_t* __restrict__ rowidx,
                                                      const double* __restrict__ cval,
                                                      const int32_t* __restrict__ a1len,
                                                      const double* __restrict__ v, const double* __restrict__ tgt,
                                                      double* __restrict__ res2, double itol2, const double* tn2,
                                                      int* inner_done, unsigned* arrive, const int* skip) {
  if (*(volatile const int*)skip) return;
  __shared__ double red[4];
  __shared__ int is_last;
  const int64_t j = blockIdx.x;
  const int64_t base = colptr[j], l1 = a1len[j];
  double sacc = 0.0;
  for (int64_t e = threadIdx.x; e < l1; e += 256) sacc += cval[base + e] * v[rowidx[base + e]];
  sacc = block_sum<256>(sacc, red);
  if (threadIdx.x == 0) {
    const double rj = tgt[j] - sacc;
    // device-scope store, then wait for it before counting the arrival: the
    // last workgroup reads every entry with device-scope loads (no fence)
    __hip_atomic_store(res2 + j, rj * rj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    is_last = __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last) return;
  double tot = 0.0;
  for (int64_t jj = threadIdx.x; jj < n; jj += 256)
    tot += __hip_atomic_load(res2 + jj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  tot = block_sum<256>(tot, red);
  if (threadIdx.x == 0) {
    *arrive = 0;
    if (tot <= itol2 * (*tn2)) *inner_done = 1;
  }
}

void launch_rk_check_csc(hipStream_t st, const ils_csr& A, const double* w, const double* s, double* v,
                         const double* tgt, double* res2, double itol2, const double* tn2, int* inner_done,
                         unsigned* arrive, const int* skip) {
  hipLaunchKernelGGL(k_sub_vec_sp, dim3(64), dim3(256), 0, st, A.p, w, s, v, skip);
  hipLaunchKernelGGL(k_rk_check_csc, dim3((unsigned)A.n), dim3(256), 0, st, A.n, (const int64_t*)A.colptr,
                     (const int32_t*)A.rowidx, (const double*)A.cval, (const int32_t*)A.a1len, (const double*)v,
                     tgt, res2, itol2, tn2, inner_done, arrive, skip);
}

}  // namespace ils
