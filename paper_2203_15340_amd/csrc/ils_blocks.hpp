// ils_blocks.hpp -- device building blocks on 64 x 64 FP64 tiles shared by the
// block Gauss-Jordan kernels and the batched solver (gfx950).
#pragma once
#include "ils_common.hpp"

namespace ils {

constexpr int kNB = 64;
// LDS row buffer of invert64: the four 16-double chunks of a row start 17
// doubles apart, so the chunks read by the four column groups fall on
// different LDS banks (a 16-double stride would put them all on one).
constexpr int kRowBuf = 4 * 17;
__device__ inline int rowbuf_at(int c) { return c + (c >> 4); }

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
__device__ inline bool invert64(double (&a)[16], int r, int g, double (*rowbuf)[kRowBuf],
                                double (*colbuf)[kNB]) {
#pragma unroll 1
  for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = kb * 16 + kk;
      const int par = kk & 1;
      if (r == k) {
#pragma unroll
        for (int v = 0; v < 16; ++v) rowbuf[par][17 * g + v] = a[v];
      }
      if (g == kb) colbuf[par][r] = a[kk];
      __syncthreads();
      double rb[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) rb[v] = rowbuf[par][17 * g + v];
      const double f = colbuf[par][r];
      const double piv = rowbuf[par][rowbuf_at(k)];
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

// LDS scratch of invert64_2d (two pivot rows and two pivot columns per
// stage, double-buffered by stage parity).
struct InvScratch2 {
  double rows[2][2][kNB];
  double cols[2][2][kNB];
};

// The inversion of invert64 with thread (ti, tj) = (t / 16, t % 16) owning the
// 4 x 4 sub-block rows 4ti.., columns 4tj.. and two pivots per barrier: a
// thread reads 2 x 4 row and 2 x 4 column values per stage instead of 16 row
// values per pivot, which is what bounds the one-row-per-thread layout (LDS
// bandwidth).  Stage K = {k, k + 1}: with P = a[K][K] and Q = P^{-1}, rows
// outside K take a[i][c] -= (a[i][K] Q) a[K][c] and a[i][K] = -a[i][K] Q,
// rows in K take Q a[K][c] and Q (block Gauss-Jordan, the same as two single
// pivots in exact arithmetic).  P must have p00 > 0 and det > 0 (the LDL^T
// pivots p00 and det / p00); otherwise every thread returns false.
__device__ inline bool invert64_2d(double (&a)[4][4], int ti, int tj, InvScratch2& S) {
  bool bad = false;
#pragma unroll 1
  for (int kq = 0; kq < 16; ++kq) {
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      const int kk = 2 * kh, k = 4 * kq + kk;
      if (ti == kq) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          S.rows[kh][0][4 * tj + j] = a[kk][j];
          S.rows[kh][1][4 * tj + j] = a[kk + 1][j];
        }
      }
      if (tj == kq) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          S.cols[kh][0][4 * ti + i] = a[i][kk];
          S.cols[kh][1][4 * ti + i] = a[i][kk + 1];
        }
      }
      __syncthreads();
      double r0[4], r1[4], c0[4], c1[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        r0[j] = S.rows[kh][0][4 * tj + j];
        r1[j] = S.rows[kh][1][4 * tj + j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        c0[i] = S.cols[kh][0][4 * ti + i];
        c1[i] = S.cols[kh][1][4 * ti + i];
      }
      const double p00 = S.rows[kh][0][k], p01 = S.rows[kh][0][k + 1];
      const double p10 = S.rows[kh][1][k], p11 = S.rows[kh][1][k + 1];
      const double det = fma(p00, p11, -p01 * p10);
      bad |= !(p00 > 0.0) || !(det > 0.0);
      const double id = recip(det);
      const double q00 = p11 * id, q01 = -p01 * id, q10 = -p10 * id, q11 = p00 * id;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool k0row = ti == kq && i == kk, k1row = ti == kq && i == kk + 1;
        double u0 = fma(c0[i], q00, c1[i] * q10), u1 = fma(c0[i], q01, c1[i] * q11);
        u0 = k0row ? 1.0 - q00 : (k1row ? -q10 : u0);
        u1 = k0row ? -q01 : (k1row ? 1.0 - q11 : u1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          double val = fma(-u0, r0[j], a[i][j]);
          val = fma(-u1, r1[j], val);
          if (j == kk) val = tj == kq ? (k0row ? 1.0 : 0.0) - u0 : val;
          if (j == kk + 1) val = tj == kq ? (k1row ? 1.0 : 0.0) - u1 : val;
          a[i][j] = val;
        }
      }
    }
  }
  return !bad;
}

}  // namespace ils
