// k_dense.hip -- streaming and MFMA kernels over the column-major ILS matrix A
// on gfx950: the column pass (A^T J b and squared column norms), the normal
// equation residual, the Gram products A1^T A1 / A2^T A2 on the matrix cores,
// and small vector/matrix helpers.
#include "ils_common.hpp"

namespace ils {

// ------------------------------------------------------------------ column pass
// One workgroup per column j: g_j = A1_(j)^T b1 - A2_(j)^T b2 (Alg. 1 step 4)
// and cn_j = ||A1_(j)||^2, the column weights of Alg. 2 steps 8 and 10.
// Non-finite entries of A or b raise kBitNonfinite.
constexpr int kColThreads = 256;

__global__ __launch_bounds__(kColThreads) void k_colpass(const double* __restrict__ A, int64_t lda,
                                                          int64_t p, int64_t q,
                                                          const double* __restrict__ b,
                                                          double* __restrict__ g,
                                                          double* __restrict__ cn, int* bits) {
  __shared__ double red[3][kColThreads / kWave];
  const int64_t j = blockIdx.x;
  const double* col = A + j * lda;
  double s1 = 0.0, s2 = 0.0, c = 0.0;
  bool ok = true;
  constexpr int U = 4;  // loads in flight per thread per round
  for (int64_t i0 = 0; i0 < p; i0 += U * kColThreads) {
    double av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + threadIdx.x + u * kColThreads;
      av[u] = i < p ? col[i] : 0.0;
      bv[u] = i < p ? b[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s1 += av[u] * bv[u];
      c += av[u] * av[u];
      ok &= isfinite(av[u]) && isfinite(bv[u]);
    }
  }
  for (int64_t i0 = p; i0 < p + q; i0 += U * kColThreads) {
    double av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + threadIdx.x + u * kColThreads;
      av[u] = i < p + q ? col[i] : 0.0;
      bv[u] = i < p + q ? b[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s2 += av[u] * bv[u];
      ok &= isfinite(av[u]) && isfinite(bv[u]);
    }
  }
  if (__any(!ok) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(bits, kBitNonfinite);
  s1 = block_sum<kColThreads>(s1, red[0]);
  s2 = block_sum<kColThreads>(s2, red[1]);
  c = block_sum<kColThreads>(c, red[2]);
  if (threadIdx.x == 0) {
    g[j] = s1 - s2;
    if (cn) cn[j] = c;
  }
}

void launch_colpass(hipStream_t s, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                    const double* b, double* g, double* cn, int* bits) {
  hipLaunchKernelGGL(k_colpass, dim3((unsigned)n), dim3(kColThreads), 0, s, A, lda, p, q, b, g, cn,
                     bits);
}

// ------------------------------------------------------------------ residual
// r = A^T J (b - A x) in two passes over A.
// Pass 1: t = b - A x, 64 rows per workgroup, the four waves split the columns
// and their partial sums are added in a fixed order.
constexpr int kResRows = 64;

__global__ __launch_bounds__(256) void k_resid_rows(const double* __restrict__ A, int64_t lda,
                                                     int64_t m, int64_t n,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ t, const int* done) {
  if (done && *done) return;
  __shared__ double part[4][kResRows];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * kResRows + lane;
  const int64_t jq = (n + 3) / 4, j0 = w * jq, j1 = j0 + jq < n ? j0 + jq : n;
  double s = 0.0;
  if (i < m) {
    const double* a = A + i;
    for (int64_t j = j0; j < j1; ++j) s += a[j * lda] * x[j];
  }
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && i < m) t[i] = b[i] - (((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
}

// Sum of x[i] y[i] over i in [i0, i1), thread share of a workgroup of NT
// threads: four loads in flight per thread per round, summed in index order.
template <int NT>
__device__ inline double strided_dot(const double* __restrict__ x, const double* __restrict__ y,
                                     int64_t i0, int64_t i1) {
  double s = 0.0;
  for (int64_t b0 = i0; b0 < i1; b0 += 4 * NT) {
    double xv[4], yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = b0 + threadIdx.x + u * NT;
      xv[u] = i < i1 ? x[i] : 0.0;
      yv[u] = i < i1 ? y[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += xv[u] * yv[u];
  }
  return s;
}

// Pass 2: r_j = A1_(j)^T t1 - A2_(j)^T t2, one workgroup per column.
__global__ __launch_bounds__(kColThreads) void k_resid_cols(const double* __restrict__ A,
                                                             int64_t lda, int64_t p, int64_t q,
                                                             const double* __restrict__ t,
                                                             double* __restrict__ r,
                                                             const int* done) {
  if (done && *done) return;
  __shared__ double red[2][kColThreads / kWave];
  const int64_t j = blockIdx.x;
  const double* col = A + j * lda;
  double s1 = 0.0, s2 = 0.0;
  s1 = strided_dot<kColThreads>(col, t, 0, p);
  s2 = strided_dot<kColThreads>(col, t, p, p + q);
  s1 = block_sum<kColThreads>(s1, red[0]);
  s2 = block_sum<kColThreads>(s2, red[1]);
  if (threadIdx.x == 0) r[j] = s1 - s2;
}

void launch_residual(hipStream_t s, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                     const double* b, const double* x, double* t, double* r, const int* done) {
  const int64_t m = p + q;
  hipLaunchKernelGGL(k_resid_rows, dim3((unsigned)((m + kResRows - 1) / kResRows)), dim3(256), 0, s,
                     A, lda, m, n, b, x, t, done);
  hipLaunchKernelGGL(k_resid_cols, dim3((unsigned)n), dim3(kColThreads), 0, s, A, lda, p, q, t, r,
                     done);
}

// ------------------------------------------------------------------ Gram (MFMA)
// G = A^T A for K rows of A (A1^T A1 or A2^T A2, Alg. 1 steps 2-3).
// Workgroup = one TM x TM tile of the lower triangle of G over one slice of
// the K rows (split-K); its four waves each own a (TM/2)^2 quadrant made of
// MFMA 16x16 blocks.  Columns of A are K-contiguous, so a TM-column x 16-row
// panel of each operand is read with 128-byte coalesced loads into registers
// one stage ahead, then written to the other half of a double-buffered LDS
// area: one barrier per stage.  Slices write partial tiles; a second kernel
// adds them in slice order (deterministic).
constexpr int kGK = 16;        // rows of A per LDS stage
constexpr int kGLd = kGK + 1;  // padded LDS row

template <typename T>
struct Mma;
template <>
struct Mma<double> {
  typedef v4d acc_t;
  __device__ static acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output element v of a lane sits at row (lane/16) + 4v, column lane%16
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mma<float> {
  typedef v4f acc_t;
  __device__ static acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element v of a lane sits at row 4*(lane/16) + v, column lane%16
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

__device__ inline void tile_of(int tile, int& ti, int& tj) {
  int r = (int)((sqrtf(8.0f * (float)tile + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= tile) ++r;
  while (r * (r + 1) / 2 > tile) --r;
  ti = r;
  tj = tile - r * (r + 1) / 2;
}

template <typename T, int TM>
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ A, int64_t lda, int64_t K,
                                              int n, int64_t klen, T* __restrict__ partials) {
  typedef typename Mma<T>::acc_t acc_t;
  constexpr int NB = TM / 32;       // 16x16 blocks per wave edge
  constexpr int NL = TM / 16;       // loads per thread per operand per stage
  __shared__ T As[2][TM][kGLd];
  __shared__ T Bs[2][TM][kGLd];
  const int tile = blockIdx.x, split = blockIdx.y;
  int ti, tj;
  tile_of(tile, ti, tj);
  const bool diag = ti == tj;
  const int64_t kbeg = (int64_t)split * klen;
  const int64_t kend = kbeg + klen < K ? kbeg + klen : K;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w >> 1) * (TM / 2), wc = (w & 1) * (TM / 2);
  const int lk = t & 15, lc = t >> 4, lr = lane & 15;
  acc_t acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[a][c] = acc_t{};
  const double* Ai = A + (int64_t)ti * TM * lda;
  const double* Aj = A + (int64_t)tj * TM * lda;
  const int ci_lim = n - ti * TM, cj_lim = n - tj * TM;
  T ra[NL], rb[NL];
  auto fetch = [&](int64_t k0) {
    const int64_t k = k0 + lk;
    const bool kin = k < kend;
#pragma unroll
    for (int r = 0; r < NL; ++r) {
      const int c = lc + 16 * r;
      ra[r] = (kin && c < ci_lim) ? (T)Ai[k + (int64_t)c * lda] : (T)0;
      if (!diag) rb[r] = (kin && c < cj_lim) ? (T)Aj[k + (int64_t)c * lda] : (T)0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int r = 0; r < NL; ++r) {
      As[buf][lc + 16 * r][lk] = ra[r];
      if (!diag) Bs[buf][lc + 16 * r][lk] = rb[r];
    }
  };
  if (kbeg < kend) {
    fetch(kbeg);
    stash(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kGK) {
    const bool more = k0 + kGK < kend;
    if (more) fetch(k0 + kGK);
    T(*Ap)[kGLd] = As[buf];
    T(*Bp)[kGLd] = diag ? As[buf] : Bs[buf];
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T fa[NB], fb[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) fa[a] = Ap[wr + a * 16 + lr][kr];
#pragma unroll
      for (int c = 0; c < NB; ++c) fb[c] = Bp[wc + c * 16 + lr][kr];
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[a][c] = Mma<T>::run(fa[a], fb[c], acc[a][c]);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  T* P = partials + ((size_t)split * gridDim.x + tile) * (TM * TM);
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int c = 0; c < NB; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + a * 16 + Mma<T>::row(lane, v);
        const int col = wc + c * 16 + lr;
        P[row * TM + col] = acc[a][c][v];
      }
}

// Sum the slices of each tile in slice order and write the tile and its
// mirror image into the full symmetric G (column-major, ldg).  One element
// per thread; the slice values are loaded together, then added in order.
template <typename T, int TM>
__global__ __launch_bounds__(256) void k_gram_finalize(const T* __restrict__ partials, int nsplit,
                                                       int ntiles, int n, double* __restrict__ G,
                                                       int64_t ldg) {
  const int tile = blockIdx.y;
  int ti, tj;
  tile_of(tile, ti, tj);
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int row = e / TM, col = e % TM;
  const int i = ti * TM + row, j = tj * TM + col;
  if (i >= n || j >= n || (ti == tj && row < col)) return;
  const T* src = partials + (size_t)tile * (TM * TM) + e;
  const size_t stride = (size_t)ntiles * (TM * TM);
  double s = 0.0;
  int sp = 0;
  for (; sp + 8 <= nsplit; sp += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[(size_t)(sp + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += (double)v[u];
  }
  for (; sp < nsplit; ++sp) s += (double)src[(size_t)sp * stride];
  G[i + (int64_t)j * ldg] = s;
  G[j + (int64_t)i * ldg] = s;
}

// Tile edge: 128 when the matrix is large enough to give the 128-tiles
// split-K work for every CU, else 64.
static int gram_tile(int64_t n) { return n >= 512 ? 128 : 64; }

static void gram_plan(int64_t n, int64_t K, int& tm, int& ntiles, int& nsplit, int64_t& klen) {
  tm = gram_tile(n);
  const int nt = (int)((n + tm - 1) / tm);
  ntiles = nt * (nt + 1) / 2;
  if (K <= 0) {
    nsplit = 1;
    klen = kGK;
    return;
  }
  const int64_t target = tm == 128 ? 512 : 1024;  // workgroups to fill 256 CUs
  int64_t want = (target + ntiles - 1) / ntiles;
  int64_t maxs = (K + 255) / 256;               // at least 256 rows per slice
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  klen = (K + want - 1) / want;
  klen = (klen + kGK - 1) / kGK * kGK;
  nsplit = (int)((K + klen - 1) / klen);
  if (nsplit < 1) nsplit = 1;
}

size_t gram_partials_size(int64_t n, int64_t K) {
  int tm, ntiles, nsplit;
  int64_t klen;
  gram_plan(n, K, tm, ntiles, nsplit, klen);
  return (size_t)ntiles * nsplit * tm * tm;
}

template <typename T, int TM>
static void gram_launch(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda, T* partials,
                        double* G, int64_t ldg, hipEvent_t mid, int ntiles, int nsplit, int64_t klen) {
  hipLaunchKernelGGL((k_gram<T, TM>), dim3(ntiles, nsplit), dim3(256), 0, s, A, lda, K, (int)n, klen,
                     partials);
  if (mid) (void)hipEventRecord(mid, s);
  hipLaunchKernelGGL((k_gram_finalize<T, TM>), dim3(TM * TM / 256, ntiles), dim3(256), 0, s, partials,
                     nsplit, ntiles, (int)n, G, ldg);
}

template <typename T>
static void gram_run(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda, T* partials,
                     double* G, int64_t ldg, hipEvent_t mid) {
  int tm, ntiles, nsplit;
  int64_t klen;
  gram_plan(n, K, tm, ntiles, nsplit, klen);
  if (tm == 128)
    gram_launch<T, 128>(s, K, n, A, lda, partials, G, ldg, mid, ntiles, nsplit, klen);
  else
    gram_launch<T, 64>(s, K, n, A, lda, partials, G, ldg, mid, ntiles, nsplit, klen);
}

void launch_gram_f64(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda,
                     double* partials, double* G, int64_t ldg, hipEvent_t mid) {
  gram_run<double>(s, K, n, A, lda, partials, G, ldg, mid);
}

void launch_gram_f32(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda,
                     float* partials, double* G, int64_t ldg, hipEvent_t mid) {
  gram_run<float>(s, K, n, A, lda, partials, G, ldg, mid);
}

// ------------------------------------------------------------------ helpers
__global__ __launch_bounds__(1024) void k_norm2(int64_t n, const double* __restrict__ v,
                                                double* __restrict__ out) {
  __shared__ double red[1024 / kWave];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s += v[i] * v[i];
  s = block_sum<1024>(s, red);
  if (threadIdx.x == 0) *out = s;
}

void launch_norm2(hipStream_t s, int64_t n, const double* v, double* out) {
  hipLaunchKernelGGL(k_norm2, dim3(1), dim3(1024), 0, s, n, v, out);
}

// Y (ncol x n, ldy) = X^T for X n x ncol (ldx), through 32x32 LDS tiles.
__global__ __launch_bounds__(256) void k_transpose(int64_t n, int64_t ncol, const double* __restrict__ X,
                                                   int64_t ldx, double* __restrict__ Y, int64_t ldy) {
  __shared__ double tileb[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + tx, j = j0 + r;
    tileb[r][tx] = (i < n && j < ncol) ? X[i + j * ldx] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + tx, i = i0 + r;
    if (i < n && j < ncol) Y[j + i * ldy] = tileb[tx][r];
  }
}

void launch_transpose(hipStream_t s, int64_t n, int64_t ncol, const double* X, int64_t ldx, double* Y,
                      int64_t ldy) {
  dim3 grid((unsigned)((n + 31) / 32), (unsigned)((ncol + 31) / 32));
  hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, n, ncol, X, ldx, Y, ldy);
}

__global__ void k_copy_cols(int64_t n, int64_t ncol, const double* __restrict__ X, int64_t ldx,
                            double* __restrict__ Y, int64_t ldy) {
  const int64_t j = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Y[i + j * ldy] = X ? X[i + j * ldx] : 0.0;
}

void launch_copy_cols(hipStream_t s, int64_t n, int64_t ncol, const double* X, int64_t ldx, double* Y,
                      int64_t ldy) {
  if (ncol <= 0 || n <= 0) return;
  unsigned gx = (unsigned)((n + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(k_copy_cols, dim3(gx, (unsigned)ncol), dim3(256), 0, s, n, ncol, X, ldx, Y, ldy);
}

void launch_fill_vec(hipStream_t s, int64_t n, const double* src, double* dst) {
  launch_copy_cols(s, n, 1, src, n, dst, n);
}

__global__ void k_eye(int64_t n, double* __restrict__ Y, int64_t ldy) {
  const int64_t j = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Y[i + j * ldy] = (i == j) ? 1.0 : 0.0;
}

void launch_eye(hipStream_t s, int64_t n, double* Y, int64_t ldy) {
  unsigned gx = (unsigned)((n + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(k_eye, dim3(gx, (unsigned)n), dim3(256), 0, s, n, Y, ldy);
}

// H = G1 - G2 (n x n, column-major, all with leading dimension ld)
__global__ void k_sub(int64_t n, const double* __restrict__ X, int64_t ldx, const double* __restrict__ Y,
                      int64_t ldy, double* __restrict__ Z, int64_t ldz) {
  const int64_t j = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Z[i + j * ldz] = X[i + j * ldx] - Y[i + j * ldy];
}

void launch_sub(hipStream_t s, int64_t n, const double* X, int64_t ldx, const double* Y, int64_t ldy,
                double* Z, int64_t ldz) {
  unsigned gx = (unsigned)((n + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(k_sub, dim3(gx, (unsigned)n), dim3(256), 0, s, n, X, ldx, Y, ldy, Z, ldz);
}

}  // namespace ils
