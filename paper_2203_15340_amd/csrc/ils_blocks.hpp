// ils_blocks.hpp -- device building blocks on 64 x 64 FP64 tiles shared by the
// block Gauss-Jordan kernels and the batched solver (gfx950).
#pragma once
#include "ils_common.hpp"

namespace ils {

constexpr int kNB = 64;

// 1/x to full double precision: hardware estimate plus two Newton steps.
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// In-place Gauss-Jordan inversion of a 64 x 64 SPD matrix held in registers
// by 256 threads: thread (r, g) = (t / 4, t % 4) owns row r, columns
// 16g..16g+15.  Before pivot k the owners of row k publish it in LDS and the
// owner of each row's column-k entry publishes that entry, so one barrier per
// pivot suffices.  Every row is updated as a <- alpha (a + beta * row_k),
// with (alpha, beta) = (1/p, 0) on the pivot row and (1, -a_rk / p) elsewhere;
// column k then takes its final value.  The pivots are those of the LDL^T
// factorisation.  Returns false (in every thread) on a pivot that is not > 0.
// The pivots run as 4 blocks of 16 unrolled steps so that every register
// index is a compile-time constant (a run-time index would send the row to
// scratch memory).
__device__ inline bool invert64(double (&a)[16], int r, int g, double (*rowbuf)[kNB],
                                double (*colbuf)[kNB]) {
#pragma unroll 1
  for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = kb * 16 + kk;
      const int par = kk & 1;
      if (r == k) {
#pragma unroll
        for (int v = 0; v < 16; ++v) rowbuf[par][16 * g + v] = a[v];
      }
      if (g == kb) colbuf[par][r] = a[kk];
      __syncthreads();
      double rb[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) rb[v] = rowbuf[par][16 * g + v];
      const double f = colbuf[par][r];
      const double piv = rowbuf[par][k];
      if (!(piv > 0.0)) return false;
      const double inv = recip(piv);
      const bool rowk = r == k;
      const double alpha = rowk ? inv : 1.0;
      const double beta = rowk ? 0.0 : -(f * inv);
      const double colval = rowk ? inv : beta;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const double val = alpha * fma(beta, rb[v], a[v]);
        a[v] = (v == kk && g == kb) ? colval : val;
      }
    }
  }
  return true;
}

}  // namespace ils
