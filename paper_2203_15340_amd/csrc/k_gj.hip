// k_gj.hip -- block Gauss-Jordan elimination on W = [G | R] for SPD G (gfx950).
//
// Algorithm 1 needs P = (A1^T A1)^{-1} only through B = P A2^T A2 and
// c = P A^T J b (steps 2-4).  Eliminating the augmented matrix
// [A1^T A1 | A2^T A2 | A^T J b] block column by block column turns it into
// [I | B | c] without storing P.  A1^T A1 is SPD (Sec. 2), so its Schur
// complements are SPD and no pivoting is needed; a pivot block that is not
// positive definite means A^T J A is not SPD either, and raises kBitNotSpd.
//
// Step k (pivot rows/columns K = [k0, k0 + nb), nb <= 64) uses two kernels:
//   k_gj_pivot : R = D^{-1} W[K, J] for every trailing column strip J, where
//                D = W[K, K]; one workgroup per 64-column strip inverts D in
//                registers and applies it on the matrix cores.  R replaces
//                W[K, J].
//   k_gj_update: W[I, J] -= W[I, K] R[K, J] for every 64-row tile I != K,
//                on the FP64 matrix cores.
// Columns left of the trailing strips are never read again.
#include "ils_common.hpp"

namespace ils {

constexpr int kNB = 64;

// Pivot kernel, one 256-thread workgroup per 64-column strip J:
//  1. D = W[K, K] (padded to 64 x 64 with the identity) is inverted in place
//     by Gauss-Jordan with the matrix held in registers: thread (r, g) owns
//     row r, columns 16g..16g+15.  Before pivot k the owners of row k publish
//     it in LDS and the owner of each row's column-k entry publishes that
//     entry, so one barrier per pivot suffices.  The pivots are those of the
//     block LDL^T factorisation, all > 0 exactly when D is SPD.
//  2. R = D^{-1} X, X = W[K, J], on the FP64 matrix cores; each wave forms a
//     32 x 32 quadrant of R^T (so that stores run down columns of W).
constexpr int kPivThreads = 256;

// 1/x to full double precision: hardware estimate plus two Newton steps.
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

__global__ __launch_bounds__(kPivThreads) void k_gj_pivot(double* __restrict__ W, int64_t ldw,
                                                          int64_t k0, int nb, int64_t c0,
                                                          int64_t ncols, int* bits) {
  __shared__ double Ds[kNB][kNB + 1];   // staging of D, later D^{-1}
  __shared__ double Xs[kNB][kNB + 1];   // Xs[c][k] = X[k][c]
  __shared__ double rowbuf[2][kNB];
  __shared__ double colbuf[2][kNB];
  if (*(volatile int*)bits) return;
  const int t = threadIdx.x;
  const int64_t cs = c0 + (int64_t)blockIdx.x * kNB;
  {
    // loads from clamped (always valid) addresses, out-of-range entries
    // replaced afterwards, so that no load sits behind a branch
    double dv[16], xv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = t + q * kPivThreads, r = e & (kNB - 1), c = e >> 6;
      const int64_t rc = r < nb ? r : nb - 1, cc = c < nb ? c : nb - 1;
      const int64_t xc = cs + c < ncols ? cs + c : ncols - 1;
      dv[q] = W[k0 + rc + (k0 + cc) * ldw];
      xv[q] = W[k0 + rc + xc * ldw];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = t + q * kPivThreads, r = e & (kNB - 1), c = e >> 6;
      Ds[r][c] = (r < nb && c < nb) ? dv[q] : (r == c ? 1.0 : 0.0);
      Xs[c][r] = (r < nb && cs + c < ncols) ? xv[q] : 0.0;
    }
  }
  __syncthreads();
  const int r = t >> 2, g = t & 3, lane = t & 63;
  double a[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) a[v] = Ds[r][16 * g + v];
#pragma unroll 1
  for (int k = 0; k < kNB; ++k) {
    const int par = k & 1;
    if (r == k) {
#pragma unroll
      for (int v = 0; v < 16; ++v) rowbuf[par][16 * g + v] = a[v];
    }
    if (g == (k >> 4)) {
      double mine = a[0];
#pragma unroll
      for (int v = 1; v < 16; ++v) mine = (v == (k & 15)) ? a[v] : mine;
      colbuf[par][r] = mine;
    }
    __syncthreads();
    double rb[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) rb[v] = rowbuf[par][16 * g + v];
    const double f = colbuf[par][r];
    const double piv = rowbuf[par][k];
    if (!(piv > 0.0)) {  // identical in every thread: the whole block leaves
      if (t == 0) atomicOr(bits, kBitNotSpd);
      return;
    }
    const double inv = recip(piv);
    const double finv = f * inv;
    const bool rowk = r == k;
    // branch-free update: both candidates are formed, then selected
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const bool colk = 16 * g + v == k;
      const double scaled = a[v] * inv;
      const double upd = fma(-finv, rb[v], a[v]);
      a[v] = rowk ? (colk ? inv : scaled) : (colk ? -finv : upd);
    }
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) Ds[r][16 * g + v] = a[v];
  __syncthreads();
  // R^T[c][i] = sum_k X[k][c] Dinv[i][k]; wave w forms the quadrant (bc, bi)
  const int w = t >> 6, cq = (w >> 1) * 32, iq = (w & 1) * 32, lr = lane & 15;
  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < kNB; kk += 4) {
    const int kr = kk + (lane >> 4);
    const double x0 = Xs[cq + lr][kr], x1 = Xs[cq + 16 + lr][kr];
    const double d0 = Ds[iq + lr][kr], d1 = Ds[iq + 16 + lr][kr];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, d0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, d1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, d0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, d1, acc[1][1], 0, 0, 0);
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = cq + x * 16 + (lane >> 4) + 4 * v, i = iq + y * 16 + lr;
        if (i < nb && cs + c < ncols) W[k0 + i + (cs + c) * ldw] = acc[x][y][v];
      }
}

// W[I, J] -= W[I, K] R[K, J].  The MFMA computes the transposed tile
// C^T[j][i] = sum_k R[k][j] W[i][k] so that a lane's four outputs run down a
// column of W (coalesced column-major stores).  All global loads of a stage
// are issued before their values are used.
__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ W, int64_t ldw, int64_t n,
                                                   int64_t k0, int nb, int64_t c0, int64_t ncols,
                                                   const int* bits) {
  __shared__ double Ws[kNB][kNB + 1];  // Ws[i][k] = W[I0 + i, k0 + k]
  __shared__ double Rs[kNB][kNB + 1];  // Rs[j][k] = W[k0 + k, J0 + j]
  if (*(volatile const int*)bits) return;
  const int64_t cs = c0 + (int64_t)blockIdx.x * kNB;
  const int64_t rs = (int64_t)blockIdx.y * kNB;
  if (rs == k0) return;  // pivot rows already hold R
  {
    double wv[16], rv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = threadIdx.x + q * 256, lo = e & (kNB - 1), hi = e >> 6;
      const int64_t wr = rs + lo < n ? rs + lo : n - 1, kc = hi < nb ? hi : nb - 1;
      const int64_t kr = lo < nb ? lo : nb - 1, jc = cs + hi < ncols ? cs + hi : ncols - 1;
      wv[q] = W[wr + (k0 + kc) * ldw];
      rv[q] = W[k0 + kr + jc * ldw];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = threadIdx.x + q * 256, lo = e & (kNB - 1), hi = e >> 6;
      Ws[lo][hi] = (rs + lo < n && hi < nb) ? wv[q] : 0.0;
      Rs[hi][lo] = (lo < nb && cs + hi < ncols) ? rv[q] : 0.0;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int jr = (w >> 1) * 32, ic = (w & 1) * 32;
  const int lr = lane & 15;
  // current values of the output tile, loaded while the MFMAs run
  double cur[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = jr + a * 16 + (lane >> 4) + 4 * v, i = ic + c * 16 + lr;
        const int64_t ir = rs + i < n ? rs + i : n - 1, jc = cs + j < ncols ? cs + j : ncols - 1;
        cur[a][c][v] = W[ir + jc * ldw];
      }
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < kNB; kk += 4) {
    const int kr = kk + (lane >> 4);
    const double a0 = Rs[jr + lr][kr], a1 = Rs[jr + 16 + lr][kr];
    const double b0 = Ws[ic + lr][kr], b1 = Ws[ic + 16 + lr][kr];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = jr + a * 16 + (lane >> 4) + 4 * v, i = ic + c * 16 + lr;
        if (rs + i < n && cs + j < ncols) W[rs + i + (cs + j) * ldw] = cur[a][c][v] - acc[a][c][v];
      }
}

void launch_gj(hipStream_t s, int64_t n, int64_t nrhs, double* W, int64_t ldw, int* bits) {
  const int64_t ncols = n + nrhs;
  const unsigned row_tiles = (unsigned)((n + kNB - 1) / kNB);
  for (int64_t k0 = 0; k0 < n; k0 += kNB) {
    const int nb = (int)(n - k0 < kNB ? n - k0 : kNB);
    const int64_t c0 = k0 + nb;
    const unsigned strips = (unsigned)((ncols - c0 + kNB - 1) / kNB);
    // with no trailing column left the pivot kernel still runs once: it tests
    // the last pivot block for positive definiteness
    hipLaunchKernelGGL(k_gj_pivot, dim3(strips > 0 ? strips : 1), dim3(kPivThreads), 0, s, W, ldw, k0,
                       nb, c0, ncols, bits);
    if (strips == 0) break;
    hipLaunchKernelGGL(k_gj_update, dim3(strips, row_tiles), dim3(256), 0, s, W, ldw, n, k0, nb, c0,
                       ncols, (const int*)bits);
  }
}

}  // namespace ils
