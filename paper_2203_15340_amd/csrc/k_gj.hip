// k_gj.hip -- block Gauss-Jordan elimination on W = [G | R] for SPD G (gfx950).
//
// Algorithm 1 needs P = (A1^T A1)^{-1} only through B = P A2^T A2 and
// c = P A^T J b (steps 2-4).  Eliminating the augmented matrix
// [A1^T A1 | A2^T A2 | A^T J b] block column by block column turns it into
// [I | B | c] without storing P.  A1^T A1 is SPD (Sec. 2), so its Schur
// complements are SPD and no pivoting is needed; a pivot block that is not
// positive definite means A^T J A is not SPD either, and raises kBitNotSpd.
//
// Step k (pivot rows/columns K = [k0, k0 + nb), nb <= 64):
//   k_gj_pivot : R = D^{-1} W[K, J] for every trailing 16-column strip J on
//                the FP64 matrix cores, with D^{-1} already inverted; R
//                replaces W[K, J].
//   k_gj_update: W[I, J] -= W[I, K] R[K, J] for every 64-row tile I != K,
//                about one workgroup per CU streaming its tiles.  Workgroup 0
//                updates the next pivot block (K+1, K+1) alone and then
//                inverts it, so the next step's pivot kernel finds D^{-1}
//                ready (one block of lookahead).
// The first pivot block is inverted by k_gj_inv0.  Columns left of the
// trailing strips are never read again.
#include "ils_common.hpp"
#include "ils_blocks.hpp"

namespace ils {

constexpr int kGjThreads = 256;

// D_0 = W[0:nb, 0:nb] -> Dinv (64 x 64, row-major), identity padding.
__global__ __launch_bounds__(kGjThreads) void k_gj_inv0(const double* __restrict__ W, int64_t ldw, int nb,
                                                        double* __restrict__ dinv, int* bits) {
  __shared__ double Ds[kNB][kLds];
  __shared__ double Es[kNB][kLds];
  __shared__ InvBlk inv;
  if (*(volatile int*)bits) return;
  const int t = threadIdx.x;
  double dv[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + q * kGjThreads, r = e & (kNB - 1), c = e >> 6;
    dv[q] = (r < nb && c < nb) ? W[r + (int64_t)c * ldw] : (r == c ? 1.0 : 0.0);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + q * kGjThreads;
    Ds[e & (kNB - 1)][e >> 6] = dv[q];
  }
  __syncthreads();
  if (!invert64_blk(&Ds[0][0], &Es[0][0], inv)) {
    if (t == 0) atomicOr(bits, kBitNotSpd);
    return;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + q * kGjThreads;
    dinv[e] = Ds[e >> 6][e & (kNB - 1)];
  }
}

// R^T[c][i] = sum_k X[k][c] Dinv[i][k] for a strip of 16 columns per
// workgroup (wave w forms rows 16w..16w+15 of R), so that a lane's four
// outputs run down a column of W.
constexpr int kPivCols = 16;

__global__ __launch_bounds__(kGjThreads) void k_gj_pivot(double* __restrict__ W, int64_t ldw,
                                                         int64_t k0, int nb, int64_t c0, int64_t ncols,
                                                         const double* __restrict__ dinv,
                                                         const int* bits) {
  __shared__ double Ds[kNB][kNB + 1];         // Ds[i][k] = Dinv[i][k]
  __shared__ double Xs[kPivCols][kNB + 1];    // Xs[c][k] = X[k][c]
  if (*(volatile const int*)bits) return;
  const int t = threadIdx.x;
  const int64_t cs = c0 + (int64_t)blockIdx.x * kPivCols;
  {
    double dv[16], xv[4];
#pragma unroll
    for (int q = 0; q < 16; ++q) dv[q] = dinv[t + q * kGjThreads];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + q * kGjThreads, lo = e & (kNB - 1), hi = e >> 6;
      xv[q] = (lo < nb && cs + hi < ncols) ? W[k0 + lo + (cs + hi) * ldw] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = t + q * kGjThreads;
      Ds[e >> 6][e & (kNB - 1)] = dv[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + q * kGjThreads;
      Xs[e >> 6][e & (kNB - 1)] = xv[q];
    }
  }
  __syncthreads();
  const int lane = t & 63, w = t >> 6, lr = lane & 15, lq = lane >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < kNB; kk += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[lr][kk + lq], Ds[16 * w + lr][kk + lq], acc, 0, 0, 0);
  const int i = 16 * w + lr;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int c = lq + 4 * v;
    if (i < nb && cs + c < ncols) W[k0 + i + (cs + c) * ldw] = acc[v];
  }
}

// W[I, J] -= W[I, K] R[K, J] over the 64 x 64 tiles (I, J), I != K.  The
// MFMA computes the transposed tile C^T[j][i] = sum_k R[k][j] W[i][k] so that
// a lane's four outputs run down a column of W (coalesced column-major
// stores).  Workgroup 0 takes the tile of the next pivot block alone and
// then inverts the updated block into dinv_next (one block of lookahead).
// The other workgroups (about one per CU) each walk a contiguous run of the
// remaining tiles; the loads of a workgroup's next tile are in flight while
// the matrix cores work on the current one, so the pass over W streams
// instead of running load, multiply and store phases in lock step.
constexpr int kUpdWgs = 256;

struct UpdTile {
  double wv[16], rv[16], cv[16];  // W[I, K] panel, R[K, J] panel, the tile itself
};

__global__ __launch_bounds__(kGjThreads) void k_gj_update(double* __restrict__ W, int64_t ldw, int64_t n,
                                                          int64_t k0, int nb, int64_t c0, int64_t ncols,
                                                          int nstrips, int row_tiles,
                                                          double* __restrict__ dinv_next, int* bits) {
  __shared__ double Ws[kNB][kNB + 1];  // Ws[i][k] = W[I0 + i, k0 + k]
  __shared__ double Rs[kNB][kNB + 1];  // Rs[j][k] = W[k0 + k, J0 + j]
  __shared__ InvBlk inv;
  if (*(volatile int*)bits) return;
  const int kt = (int)(k0 / kNB);
  const bool has_next = k0 + kNB < n;
  // tile list: the non-pivot row tiles in order, nstrips tiles each; the
  // lookahead tile (kt + 1, strip 0) sits at list position kt * nstrips and
  // is swapped with position 0
  const int ntile = (row_tiles - 1) * nstrips;
  const int pla = kt * nstrips;
  auto tile_at = [&](int L, int64_t& rs, int64_t& cs) {
    if (has_next) L = L == 0 ? pla : (L == pla ? 0 : L);
    const int rt = L / nstrips;
    rs = (int64_t)(rt >= kt ? rt + 1 : rt) * kNB;
    cs = c0 + (int64_t)(L % nstrips) * kNB;
  };
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int jr = (w >> 1) * 32, ic = (w & 1) * 32;
  const int lr = lane & 15;
  // with_w: also the W[I, K] panel (skipped when the previous tile had the
  // same row block, whose panel is still in LDS)
  auto load = [&](int64_t rs, int64_t cs, UpdTile& T, bool with_w) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = threadIdx.x + q * kGjThreads, lo = e & (kNB - 1), hi = e >> 6;
      if (with_w) T.wv[q] = (rs + lo < n && hi < nb) ? W[rs + lo + (k0 + hi) * ldw] : 0.0;
      T.rv[q] = (lo < nb && cs + hi < ncols) ? W[k0 + lo + (cs + hi) * ldw] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = jr + a * 16 + (lane >> 4) + 4 * v, i = ic + c * 16 + lr;
          T.cv[(a * 2 + c) * 4 + v] = (rs + i < n && cs + j < ncols) ? W[rs + i + (cs + j) * ldw] : 0.0;
        }
  };
  auto stash = [&](const UpdTile& T, bool with_w) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = threadIdx.x + q * kGjThreads, lo = e & (kNB - 1), hi = e >> 6;
      if (with_w) Ws[lo][hi] = T.wv[q];
      Rs[hi][lo] = T.rv[q];
    }
  };
  // C = tile - W[I, K] R[K, J], kept in cv; columns j >= jmin of the tile
  // are written to W
  auto multiply_store = [&](int64_t rs, int64_t cs, UpdTile& T, int jmin) {
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
          const double val = T.cv[(a * 2 + c) * 4 + v] - acc[a][c][v];
          T.cv[(a * 2 + c) * 4 + v] = val;
          if (j >= jmin && rs + i < n && cs + j < ncols) W[rs + i + (cs + j) * ldw] = val;
        }
  };
  if (has_next && blockIdx.x == 0) {
    // the next pivot block: update, then invert (identity outside it); no
    // later step reads the block itself, only its inverse, so only the
    // tile's columns right of it (a short last block) go back to W
    int64_t rs, cs;
    tile_at(0, rs, cs);
    const int nbn = (int)(n - rs < kNB ? n - rs : kNB);
    UpdTile T;
    load(rs, cs, T, true);
    stash(T, true);
    __syncthreads();
    multiply_store(rs, cs, T, nbn);
    __syncthreads();  // everyone is done reading Ws
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = jr + a * 16 + (lane >> 4) + 4 * v, i = ic + c * 16 + lr;
          Ws[i][j] = (i < nbn && j < nbn) ? T.cv[(a * 2 + c) * 4 + v] : (i == j ? 1.0 : 0.0);
        }
    __syncthreads();
    if (!invert64_blk(&Ws[0][0], &Rs[0][0], inv)) {
      if (threadIdx.x == 0) atomicOr(bits, kBitNotSpd);
      return;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = threadIdx.x + q * kGjThreads;
      dinv_next[e] = Ws[e >> 6][e & (kNB - 1)];
    }
    return;
  }
  // the other tiles: workgroup b >= first takes a contiguous run of list
  // positions (mostly one row block, so the W[I, K] panel is loaded once per
  // row), two register sets in turn
  const int first = has_next ? 1 : 0;
  const int nw = (int)gridDim.x - first;
  if (nw <= 0) return;
  const int cnt = ntile - first;
  const int chunk = (cnt + nw - 1) / nw;
  int L = first + ((int)blockIdx.x - first) * chunk;
  const int Lend = L + chunk < ntile ? L + chunk : ntile;
  if (L >= Lend) return;
  UpdTile X, Y;
  int64_t rx, cx, ry, cy, wrow = -1;
  tile_at(L, rx, cx);
  load(rx, cx, X, true);
  while (true) {
    stash(X, rx != wrow);
    wrow = rx;
    const int L1 = L + 1;
    if (L1 < Lend) {
      tile_at(L1, ry, cy);
      load(ry, cy, Y, ry != rx);
    }
    __syncthreads();
    multiply_store(rx, cx, X, 0);
    __syncthreads();  // Ws, Rs free again
    if (L1 >= Lend) break;
    stash(Y, ry != wrow);
    wrow = ry;
    L = L1 + 1;
    if (L < Lend) {
      tile_at(L, rx, cx);
      load(rx, cx, X, rx != ry);
    }
    __syncthreads();
    multiply_store(ry, cy, Y, 0);
    __syncthreads();
    if (L >= Lend) break;
  }
}

size_t gj_dinv_size() { return 2 * kNB * kNB; }

void launch_gj(hipStream_t s, int64_t n, int64_t nrhs, double* W, int64_t ldw, double* dinv, int* bits) {
  const int64_t ncols = n + nrhs;
  const int row_tiles = (int)((n + kNB - 1) / kNB);
  hipLaunchKernelGGL(k_gj_inv0, dim3(1), dim3(kGjThreads), 0, s, (const double*)W, ldw,
                     (int)(n < kNB ? n : kNB), dinv, bits);
  int step = 0;
  for (int64_t k0 = 0; k0 < n; k0 += kNB, ++step) {
    const int nb = (int)(n - k0 < kNB ? n - k0 : kNB);
    const int64_t c0 = k0 + nb;
    const int strips = (int)((ncols - c0 + kNB - 1) / kNB);
    if (strips <= 0) break;
    double* dcur = dinv + (step & 1) * kNB * kNB;
    double* dnext = dinv + ((step + 1) & 1) * kNB * kNB;
    const int pstrips = (int)((ncols - c0 + kPivCols - 1) / kPivCols);
    hipLaunchKernelGGL(k_gj_pivot, dim3(pstrips), dim3(kGjThreads), 0, s, W, ldw, k0, nb, c0, ncols,
                       (const double*)dcur, (const int*)bits);
    const int ntile = (row_tiles - 1) * strips;
    if (ntile > 0) {
      const int wgs = ntile < kUpdWgs ? ntile : kUpdWgs;
      hipLaunchKernelGGL(k_gj_update, dim3(wgs), dim3(kGjThreads), 0, s, W, ldw, n, k0, nb, c0, ncols, strips,
                         row_tiles, dnext, bits);
    }
  }
}

}  // namespace ils
