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
//                D = W[K, K]; one workgroup per 64-column strip, the small
//                elimination runs in LDS.  R replaces W[K, J].
//   k_gj_update: W[I, J] -= W[I, K] R[K, J] for every 64-row tile I != K,
//                on the FP64 matrix cores.
// Columns left of the trailing strips are never read again.
#include "ils_common.hpp"

namespace ils {

constexpr int kNB = 64;

__global__ __launch_bounds__(256) void k_gj_pivot(double* __restrict__ W, int64_t ldw, int64_t k0,
                                                  int nb, int64_t c0, int64_t ncols, int* bits) {
  __shared__ double D[kNB][kNB + 1];
  __shared__ double X[kNB][kNB + 1];
  if (*(volatile int*)bits) return;
  const int64_t cs = c0 + (int64_t)blockIdx.x * kNB;
  for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
    const int r = e % kNB, c = e / kNB;
    D[r][c] = (r < nb && c < nb) ? W[k0 + r + (k0 + c) * ldw] : (r == c ? 1.0 : 0.0);
    X[r][c] = (r < nb && cs + c < ncols) ? W[k0 + r + (cs + c) * ldw] : 0.0;
  }
  __syncthreads();
  for (int i = 0; i < nb; ++i) {
    const double piv = D[i][i];
    if (!(piv > 0.0)) {  // same value in every thread: the whole block leaves
      if (threadIdx.x == 0) atomicOr(bits, kBitNotSpd);
      return;
    }
    const double inv = 1.0 / piv;
    __syncthreads();
    for (int c = threadIdx.x; c < 2 * kNB; c += 256) {
      if (c < kNB) {
        if (c > i) D[i][c] *= inv;
      } else {
        X[i][c - kNB] *= inv;
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kNB * 2 * kNB; e += 256) {
      const int r = e % kNB, c = e / kNB;
      if (r == i || r >= nb) continue;
      const double f = D[r][i];
      if (c < kNB) {
        if (c > i) D[r][c] -= f * D[i][c];
      } else {
        X[r][c - kNB] -= f * X[i][c - kNB];
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
    const int r = e % kNB, c = e / kNB;
    if (r < nb && cs + c < ncols) W[k0 + r + (cs + c) * ldw] = X[r][c];
  }
}

// W[I, J] -= W[I, K] R[K, J].  The MFMA computes the transposed tile
// C^T[j][i] = sum_k R[k][j] W[i][k] so that a lane's four outputs run down a
// column of W (coalesced column-major stores).
__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ W, int64_t ldw, int64_t n,
                                                   int64_t k0, int nb, int64_t c0, int64_t ncols,
                                                   const int* bits) {
  __shared__ double Ws[kNB][kNB + 1];  // Ws[i][k] = W[I0 + i, k0 + k]
  __shared__ double Rs[kNB][kNB + 1];  // Rs[j][k] = W[k0 + k, J0 + j]
  if (*(volatile const int*)bits) return;
  const int64_t cs = c0 + (int64_t)blockIdx.x * kNB;
  const int64_t rs = (int64_t)blockIdx.y * kNB;
  if (rs == k0) return;  // pivot rows already hold R
  for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
    const int i = e % kNB, k = e / kNB;
    Ws[i][k] = (rs + i < n && k < nb) ? W[rs + i + (k0 + k) * ldw] : 0.0;
    const int kk = e % kNB, j = e / kNB;
    Rs[j][kk] = (kk < nb && cs + j < ncols) ? W[k0 + kk + (cs + j) * ldw] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int jr = (w >> 1) * 32, ic = (w & 1) * 32;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = v4d{0.0, 0.0, 0.0, 0.0};
  const int lr = lane & 15;
#pragma unroll 4
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
        const int j = jr + a * 16 + (lane >> 4) + 4 * v;
        const int i = ic + c * 16 + lr;
        if (rs + i < n && cs + j < ncols) W[rs + i + (cs + j) * ldw] -= acc[a][c][v];
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
    hipLaunchKernelGGL(k_gj_pivot, dim3(strips > 0 ? strips : 1), dim3(256), 0, s, W, ldw, k0, nb, c0,
                       ncols, bits);
    if (strips == 0) break;
    hipLaunchKernelGGL(k_gj_update, dim3(strips, row_tiles), dim3(256), 0, s, W, ldw, n, k0, nb, c0,
                       ncols, (const int*)bits);
  }
}

}  // namespace ils
