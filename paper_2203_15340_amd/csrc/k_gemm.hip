// k_gemm.hip -- C = alpha * X^T S Y + beta * C0 on the FP64 matrix cores.
//
// The one general product of the multi-right-hand-side SP solve:
//   A^T J B  (X = A, Y = B, S = J = diag(I_p, -I_q): rows k >= p of Y enter
//             negated; the right-hand sides of (Sec12) for many b at once),
//   B X_k    (X = B^T, Y = X_k: the SP update of Alg. 1 step 6 for many x),
//   H X_k    (X = H = A^T J A, symmetric: residuals for the RR stop test).
// X is K x M and Y is K x N, both column-major with K contiguous, so both
// operands stream K-contiguous columns like the Gram kernel.  Workgroup =
// one 64 x 64 tile of C, four waves of 32 x 32 made of MFMA 16 x 16 blocks;
// 16-row panels are prefetched into registers one stage ahead and written to
// a double-buffered LDS area (one barrier per stage).
//
// An optional column mask freezes columns: where active[j] == 0, C[:, j]
// receives keep[:, j] instead (a converged right-hand side keeps its
// iterate), and tiles whose columns are all frozen skip the product.
#include "ils_common.hpp"

namespace ils {

constexpr int kMK = 16;        // K rows per stage
constexpr int kMLd = kMK + 1;  // padded LDS row
constexpr int kMT = 64;        // tile edge

__global__ __launch_bounds__(256) void k_gemm_tn(GemmTnArgs g) {
  __shared__ double Xs[2][kMT][kMLd];
  __shared__ double Ys[2][kMT][kMLd];
  const int64_t mt = (g.M + kMT - 1) / kMT;
  const int64_t ti = blockIdx.x % mt, tj = blockIdx.x / mt;
  const int64_t i0 = ti * kMT, j0 = tj * kMT;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int lk = t & 15, lc = t >> 4, lr = lane & 15;
  const int ilim = (int)(g.M - i0 < kMT ? g.M - i0 : kMT);
  const int jlim = (int)(g.N - j0 < kMT ? g.N - j0 : kMT);

  int any = 1;
  if (g.active) {
    const int j = t & 63;
    any = (t < 64 && j < jlim) ? g.active[j0 + j] : 0;
    any = __syncthreads_or(any);
  }
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = v4d{};

  if (any) {
    const double* Xi = g.X + i0 * g.ldx;
    const double* Yj = g.Y + j0 * g.ldy;
    double rx[4], ry[4];
    auto fetch = [&](int64_t k0) {
      const int64_t k = k0 + lk;
      const bool kin = k < g.K;
      const double sg = k < g.kneg ? 1.0 : -1.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = lc + 16 * r;
        rx[r] = (kin && c < ilim) ? Xi[k + (int64_t)c * g.ldx] : 0.0;
        ry[r] = (kin && c < jlim) ? sg * Yj[k + (int64_t)c * g.ldy] : 0.0;
      }
    };
    auto stash = [&](int buf) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Xs[buf][lc + 16 * r][lk] = rx[r];
        Ys[buf][lc + 16 * r][lk] = ry[r];
      }
    };
    fetch(0);
    stash(0);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = 0; k0 < g.K; k0 += kMK) {
      const bool more = k0 + kMK < g.K;
      if (more) fetch(k0 + kMK);
#pragma unroll
      for (int kk = 0; kk < kMK; kk += 4) {
        const int kr = kk + (lane >> 4);
        double fa[2], fb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) fa[a] = Xs[buf][wr + a * 16 + lr][kr];
#pragma unroll
        for (int c = 0; c < 2; ++c) fb[c] = Ys[buf][wc + c * 16 + lr][kr];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[c], acc[a][c], 0, 0, 0);
      }
      if (more) stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // epilogue: output element v of a lane sits at row (lane/16) + 4v, column lane%16
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int jl = wc + c * 16 + lr;
    if (jl >= jlim) continue;
    const int64_t j = j0 + jl;
    const bool live = !g.active || g.active[j];
    if (!live && !g.keep) continue;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int il = wr + a * 16 + (lane >> 4) + 4 * v;
        if (il >= ilim) continue;
        const int64_t i = i0 + il;
        double val;
        if (live) {
          val = g.alpha * acc[a][c][v];
          if (g.beta != 0.0) val += g.beta * g.C0[i + j * g.ldc0];
        } else {
          val = g.keep[i + j * g.ldkeep];
        }
        g.C[i + j * g.ldc] = val;
      }
  }
}

void launch_gemm_tn(hipStream_t s, const GemmTnArgs& g) {
  if (g.M <= 0 || g.N <= 0) return;
  const int64_t tiles = ((g.M + kMT - 1) / kMT) * ((g.N + kMT - 1) / kMT);
  hipLaunchKernelGGL(k_gemm_tn, dim3((unsigned)tiles), dim3(256), 0, s, g);
}

}  // namespace ils
