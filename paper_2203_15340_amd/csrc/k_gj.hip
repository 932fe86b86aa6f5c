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
//
// Up to kFlowMaxRows block rows (n <= 2048) the same items run as one
// dataflow launch instead (k_gj_flow below): no step waits for the whole
// previous step, only for the tiles it reads, so the chain of pivot-block
// inversions is the critical path rather than one launch pair per step.
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

// ------------------------------------------------------------- dataflow form
// For n up to kFlowMaxRows blocks the whole elimination is one persistent
// launch: workgroups take work items from a ticket counter and each item
// waits, by polling counters in device memory, only for the items whose
// output it reads.  Items of step k (pivot block K = block row k):
//   L_k        (k + 1 < R) update the next pivot block (k+1, k+1) with step
//              k's pivot rows, formed here from D_k^{-1} (the block is
//              C - X^T D_k^{-1} X with X = W[K, k+1], C = W[k+1, k+1]: a
//              symmetric Schur complement), and invert it; the chain
//              L_0 -> L_1 -> ... is the critical path, run in turn by the
//              workgroup holding L_0's ticket, each inverse kept in its LDS;
//   P(k, j)    R_j = D_k^{-1} W[K, j] in place, for every trailing strip j;
//   U(k, i, j) W[i, j] -= W[i, K] R_j for every row block i != k;
//   PC(k)      when strip k+2 is a whole block of the matrix part, P(k, k+2)
//              together with U(k, k+1, k+2) and U(k, k+2, k+2): the two tiles
//              L_{k+1} reads, formed as soon as D_k^{-1} is out (their
//              multipliers W[k+1, K] and W[k+2, K] taken, by the symmetry of
//              the Schur complement, as the transposes of W[K, k+1] and
//              W[K, k+2]), so the chain need not wait for the rest of the
//              strip; the two U items then have nothing to do.
// Strips are the 64-column blocks of W (the last pivot block may be short,
// then its strip also holds right-hand-side columns).  Counters:
//   tcnt[i][j]  steps that have updated tile (i, j) (block row i, strip j):
//               every step k < j writes every tile of strip j once, except
//               the pivot block (k+1, k+1) of L_k, so an item that needs the
//               tile as of step k - 1 waits for tcnt >= k,
//   cnt[k][j]   items of step k done with strip j (R of them, R - 1 for strip
//               k+1, whose row k+1 belongs to L_k): U(k, k-1, j) overwrites the
//               previous pivot row's tile, which every item of step k - 1 in
//               strip j reads, so it waits for all of them,
//   pdone[k][j] P(k, j) done,  dflag[k] D_k^{-1} published,
//   lflag[k]    L_k (and PC(k)) have read W[K, k+1], which P(k, k+1) then
//               overwrites.
// Tickets are issued in step order (within a step: L_k, PC(k), the P items,
// then the U items strip by strip; in a strip, the rows below the pivot
// first).  An item only waits for items with smaller tickets, which are held
// by running workgroups, or for the chain's inverses and flags; the chain's
// link k waits only for items of step k - 1, which need nothing from it
// beyond D_{k-1}^{-1}; so every wait ends.  A bounded spin still raises
// kBitStall rather than hanging if one did not.
constexpr int kFlowMaxRows = 32;
constexpr int kFlowOcc = 1;  // workgroups per CU
constexpr int kFlowWgs = 256 * kFlowOcc;
constexpr int kSpinLimit = 1 << 22;

struct GjFlow {
  double* W;
  int64_t ldw, n, ncols;
  int R, S;
  double* dinv;  // R blocks of 64 x 64, row-major
  int* tcnt;     // R x S
  int* cnt;      // R x S
  int* pdone;    // R x S
  int* dflag;    // R
  int* lflag;    // R
  unsigned* ticket;
  int* bits;
  GjCombine pre;  // optional right-hand-side column formed first (see launch_gj)
  GjExtras ex;    // optional loop-state reset and row-major copy (see launch_gj)
};

struct FlowStep {
  int nb, j0, nP, nI;
  int64_t c0;
  bool hasL;
};

__device__ inline FlowStep flow_step(const GjFlow& a, int k) {
  FlowStep f;
  const int64_t k0 = (int64_t)k * kNB;
  f.nb = (int)(a.n - k0 < kNB ? a.n - k0 : kNB);
  f.c0 = k0 + f.nb;
  f.j0 = (int)(f.c0 / kNB);
  f.hasL = k + 1 < a.R;
  f.nP = f.c0 < a.ncols ? a.S - f.j0 : 0;
  const int nU = f.nP > 0 ? (a.R - 1) * f.nP - (f.hasL ? 1 : 0) : 0;
  f.nI = (f.hasL ? 1 : 0) + f.nP + nU;
  return f;
}

// whether step k has a PC item (see above)
__device__ inline bool flow_pc(const GjFlow& a, int k) { return (int64_t)(k + 3) * kNB <= a.n; }

// the value of tcnt[i][j] once tile (i, j) is as of step k - 1 (the pivot
// block (j, j) is not written at step j - 1)
__device__ inline int tile_need(int i, int j, int k) { return (i == j && k >= j) ? j - 1 : k; }
__device__ inline int* tile_cnt(const GjFlow& a, int i, int j) { return a.tcnt + i * a.S + j; }

// items of step k that finish with strip j (see above)
__device__ inline int flow_target(const GjFlow& a, int k, int j) {
  return (k + 1 < a.R && j == k + 1) ? a.R - 1 : a.R;
}

// Thread 0 polls until *p >= tp and *q >= tq (both read in one round trip).
__device__ inline bool flow_wait2(const int* p, int tp, const int* q, int tq, int* bits) {
  for (int spin = 0;; ++spin) {
    const int vp = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int vq = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (vp >= tp && vq >= tq) return true;
    if (__hip_atomic_load(bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (spin >= kSpinLimit) {
      atomicOr(bits, kBitStall);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Thread 0 polls until *p >= target; false if the bits were raised meanwhile.
__device__ inline bool flow_wait(const int* p, int target, int* bits) {
  for (int spin = 0;; ++spin) {
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) return true;
    if (__hip_atomic_load(bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (spin >= kSpinLimit) {
      atomicOr(bits, kBitStall);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// W and the inverses are read and written inside the launch with device-scope
// relaxed atomic loads and stores: those bypass the non-coherent caches
// (each XCD has its own L2), so no cache write-back or invalidation is needed
// around a hand-over.  A producer waits until its stores are acknowledged
// (vmcnt 0), then one thread counts.
__device__ inline double ald(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void ast(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void wait_stores() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's stores have completed
}
__device__ inline void flow_signal(int* p) {
  wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kGjThreads, kFlowOcc) void k_gj_flow(GjFlow a) {
  __shared__ double As[kNB][kNB + 1];  // A operand: As[i][k]
  __shared__ double Bs[kNB][kNB + 1];  // B operand: Bs[j][k]
  __shared__ double Ds[kNB][kNB + 1];  // L_k: the next pivot block, then its inverse
  __shared__ InvBlk inv;
  __shared__ int s_tk, s_ok;
  if (__hip_atomic_load(a.bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int jr = (w >> 1) * 32, ic = (w & 1) * 32, lr = lane & 15;
  double* W = a.W;
  const int64_t ldw = a.ldw, n = a.n, ncols = a.ncols;
  // 64 x 64 block of W at (r0, c0) into registers (e = t + 256 q: row e & 63,
  // column e >> 6); rows >= rmax, columns outside [cmin, cmax) and columns
  // >= c0 + kmax read as zero
  auto load_tile = [&](double (&v)[16], int64_t r0, int64_t c0, int64_t rmax, int64_t cmin, int64_t cmax) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = t + q * kGjThreads, lo = e & (kNB - 1), hi = e >> 6;
      const int64_t r = r0 + lo, c = c0 + hi;
      v[q] = (r < rmax && c >= cmin && c < cmax) ? ald(W + r + c * ldw) : 0.0;
    }
  };
  // the same block in the product's output layout (C^T lanes)
  auto load_out = [&](double (&v)[16], int64_t r0, int64_t c0, int64_t rmax, int64_t cmin, int64_t cmax) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = jr + x * 16 + (lane >> 4) + 4 * u, i = ic + y * 16 + lr;
          const int64_t r = r0 + i, c = c0 + j;
          v[(x * 2 + y) * 4 + u] = (r < rmax && c >= cmin && c < cmax) ? ald(W + r + c * ldw) : 0.0;
        }
  };
  auto store_out = [&](const double (&v)[16], int64_t r0, int64_t c0, int64_t rmax, int64_t cmin, int64_t cmax) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = jr + x * 16 + (lane >> 4) + 4 * u, i = ic + y * 16 + lr;
          const int64_t r = r0 + i, c = c0 + j;
          if (r < rmax && c >= cmin && c < cmax) ast(W + r + c * ldw, v[(x * 2 + y) * 4 + u]);
        }
  };
  // the last step's final tiles also go row-major into ex.bt (columns
  // [bcol0, bcol0 + nbt)), through As: every wave is past its product
  auto store_bt = [&](const double (&v)[16], int64_t r0, int64_t c0) {
    if (c0 + kNB <= a.ex.bcol0 || c0 >= a.ex.bcol0 + a.ex.nbt) return;
    __syncthreads();
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int u = 0; u < 4; ++u) As[ic + y * 16 + lr][jr + x * 16 + (lane >> 4) + 4 * u] = v[(x * 2 + y) * 4 + u];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = t + q * kGjThreads, i = e >> 6, j = e & (kNB - 1);
      const int64_t r = r0 + i, c = c0 + j;
      if (r < n && c >= a.ex.bcol0 && c < a.ex.bcol0 + a.ex.nbt) a.ex.bt[(c - a.ex.bcol0) + r * a.ex.ldbt] = As[i][j];
    }
  };
  // tile (A operand) As[i][k] = v(i, k); (B operand) Bs[j][k] = v(k, j)
  auto stash_a = [&](const double (&v)[16]) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = t + q * kGjThreads;
      As[e & (kNB - 1)][e >> 6] = v[q];
    }
  };
  auto stash_b = [&](const double (&v)[16]) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = t + q * kGjThreads;
      Bs[e >> 6][e & (kNB - 1)] = v[q];
    }
  };
  auto stash_dinv = [&](const double* D) {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = ald(D + t + q * kGjThreads);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = t + q * kGjThreads;
      As[e >> 6][e & (kNB - 1)] = v[q];
    }
  };
  // acc (output layout) = A B over the full 64-deep contraction, A from Ao
  // (Ao[i][k] = A(i, k)), B from Bs
  auto product_a = [&](double (&acc)[16], const double (*Ao)[kNB + 1]) {
    v4d c4[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) c4[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < kNB; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double b0 = Bs[jr + lr][kr], b1 = Bs[jr + 16 + lr][kr];
      const double a0 = Ao[ic + lr][kr], a1 = Ao[ic + 16 + lr][kr];
      c4[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, c4[0][0], 0, 0, 0);
      c4[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, c4[0][1], 0, 0, 0);
      c4[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, c4[1][0], 0, 0, 0);
      c4[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, c4[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[(x * 2 + y) * 4 + u] = c4[x][y][u];
  };
  auto product = [&](double (&acc)[16]) { product_a(acc, As); };
  // thread 0 runs the waits; every thread learns the outcome
  auto finish_wait = [&](bool ok) {
    if (t == 0) s_ok = ok;
    __syncthreads();
    const bool r = s_ok;
    return r;
  };

  int k = 0;
  int base = 0;
  FlowStep f = flow_step(a, 0);
  for (;;) {
    __syncthreads();  // LDS of the previous item free
    if (t == 0) s_tk = (int)atomicAdd(a.ticket, 1u);
    __syncthreads();
    const int tk = s_tk;
    while (k < a.R && tk >= base + f.nI) {
      base += f.nI;
      ++k;
      if (k < a.R) f = flow_step(a, k);
    }
    if (k >= a.R) break;
    int u = tk - base;
    const int64_t k0 = (int64_t)k * kNB;
    const int R = a.R;
    if (f.hasL && u == 0) {
      // ---- the chain: L_0, L_1, ... in this one workgroup, each inverse kept in
      // LDS for the next link (the later L_k tickets have nothing to do)
      if (k > 0) continue;
      for (int kc = 0; kc + 1 < R; ++kc) {
        // L_k: D_{k+1} = W[k+1, k+1] - W[k+1, K] D_k^{-1} W[K, k+1], inverted
        const int k = kc;
        const int64_t k0 = (int64_t)k * kNB, k1 = k0 + kNB;
        const int nbn = (int)(n - k1 < kNB ? n - k1 : kNB);
        // the Schur complement is symmetric, so M = W[k+1, K] is taken as X^T:
        // both tiles read here lie in strip k + 1
        bool ok = true;
        if (t == 0 && k >= 1)
          ok = flow_wait2(tile_cnt(a, k, k + 1), k, tile_cnt(a, k + 1, k + 1), k, a.bits);
        if (!finish_wait(ok)) break;
        double xv[16], cv[16];
        load_tile(xv, k0, k1, k0 + kNB, k1, ncols);  // X = W[K, k+1]
        load_out(cv, k1, k1, n, k1, ncols);          // C = W[k+1, k+1]
        // the first look at D_k^{-1}'s flag goes out with the tile loads
        int dseen = 0;
        if (t == 0 && k == 0) dseen = __hip_atomic_load(a.dflag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        stash_b(xv);                                 // X has been read
        __syncthreads();
        if (t == 0) {
          __hip_atomic_fetch_add(a.lflag + k, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (k == 0) ok = dseen >= 1 || flow_wait(a.dflag, 1, a.bits);
        }
        if (!finish_wait(ok)) break;
        double acc[16];
        if (k == 0) {
          stash_dinv(a.dinv);
          __syncthreads();
          product(acc);  // R = D_0^{-1} X
        } else {
          product_a(acc, Ds);  // R = D_k^{-1} X, D_k^{-1} left in Ds by the previous link
        }
        __syncthreads();
        // As[i][k] = M(i, k) = X(k, i)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int e = t + q * kGjThreads;
          As[e >> 6][e & (kNB - 1)] = xv[q];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int j = jr + x * 16 + (lane >> 4) + 4 * q, i = ic + y * 16 + lr;
              Bs[j][i] = acc[(x * 2 + y) * 4 + q];
              Ds[i][j] = cv[(x * 2 + y) * 4 + q];  // C, row-major
            }
        __syncthreads();
        bool inv_ok;
        double(*Dinv)[kNB + 1];
        if (nbn == kNB) {
          // D = C - M R is symmetric: its lower 16 x 16 blocks are formed and
          // mirrored, and wave 0 takes block (0, 0) alone and inverts it while
          // waves 1-3 form the other nine
          const int li = lane & 15, lg = lane >> 4;
          auto block_d = [&](int bi, int bj) {
            v4d d = ld16(&Ds[16 * bi][16 * bj], kLds, lane);
#pragma unroll
            for (int kk = 0; kk < kNB; kk += 4) {
              const int kr = kk + lg;
              d = __builtin_amdgcn_mfma_f64_16x16x4f64(-As[16 * bi + li][kr], Bs[16 * bj + li][kr], d, 0, 0, 0);
            }
            return d;
          };
          if (w == 0) {
            st16(&Ds[0][0], kLds, block_d(0, 0), lane);
            __threadfence_block();
            double av[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) av[c] = Ds[li][4 * lg + c];
            const bool okl = leaf_inv16(av, lane);
#pragma unroll
            for (int c = 0; c < 4; ++c) inv.x[li][4 * lg + c] = av[c];
            if (lane == 0) inv.bad = okl ? 0 : 1;
          } else {
            // (1,0) (1,1) (2,0) | (2,1) (2,2) (3,0) | (3,1) (3,2) (3,3)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              const int e = 3 * (w - 1) + q;
              const int bi = e < 2 ? 1 : (e < 5 ? 2 : 3);
              const int bj = e - (bi == 1 ? 0 : (bi == 2 ? 2 : 5));
              const v4d d = block_d(bi, bj);
              st16(&Ds[16 * bi][16 * bj], kLds, d, lane);
              if (bi != bj) {
#pragma unroll
                for (int u = 0; u < 4; ++u) Ds[16 * bj + li][16 * bi + lg + 4 * u] = d[u];
              }
            }
          }
          __syncthreads();
          if (w == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) Bs[li][4 * lg + c] = inv.x[li][4 * lg + c];
          }
          __syncthreads();
          inv_ok = invert64_steps(&Ds[0][0], &Bs[0][0], inv);
          Dinv = Ds;
        } else {
          product(acc);  // M R
#pragma unroll
          for (int q = 0; q < 16; ++q) cv[q] -= acc[q];
          // right-hand-side columns sharing the short last block's strip
          store_out(cv, k1, k1, n, k1 + nbn, ncols);
          __syncthreads();
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int j = jr + x * 16 + (lane >> 4) + 4 * q, i = ic + y * 16 + lr;
                As[i][j] = (i < nbn && j < nbn) ? cv[(x * 2 + y) * 4 + q] : (i == j ? 1.0 : 0.0);
              }
          __syncthreads();
          inv_ok = invert64_blk(&As[0][0], &Bs[0][0], inv);
          Dinv = As;
        }
        if (!inv_ok) {
          if (t == 0) atomicOr(a.bits, kBitNotSpd);
          break;
        }
        double* dn = a.dinv + (int64_t)(k + 1) * kNB * kNB;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int e = t + q * kGjThreads;
          ast(dn + e, Dinv[e >> 6][e & (kNB - 1)]);
        }
        flow_signal(a.dflag + k + 1);  // also: every wave has read Dinv
      }
      continue;
    }
    if (f.hasL) --u;
    const bool pc = flow_pc(a, k);
    if (pc && u == 0) {
      // ---- PC(k): R = D_k^{-1} W[K, k+2] in place, then
      // W[k+1, k+2] -= X^T R and W[k+2, k+2] -= W[K, k+2]^T R (X = W[K, k+1])
      const int64_t k1 = k0 + kNB, k2 = k1 + kNB;
      bool ok = true;
      if (t == 0 && k >= 1) {
        ok = flow_wait(tile_cnt(a, k, k + 1), k, a.bits) && flow_wait(tile_cnt(a, k, k + 2), k, a.bits) &&
             flow_wait(tile_cnt(a, k + 1, k + 2), k, a.bits) && flow_wait(tile_cnt(a, k + 2, k + 2), k, a.bits);
      }
      if (!finish_wait(ok)) continue;
      double xv[16], pv[16], c1[16], c2[16];
      load_tile(xv, k0, k1, k0 + kNB, k1, ncols);  // X = W[K, k+1]
      load_tile(pv, k0, k2, k0 + kNB, k2, ncols);  // W[K, k+2]
      load_out(c1, k1, k2, n, k2, ncols);          // W[k+1, k+2]
      load_out(c2, k2, k2, n, k2, ncols);          // W[k+2, k+2]
      int dseen = 0;
      if (t == 0) dseen = __hip_atomic_load(a.dflag + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // Ds[i][k] = X(k, i): the multiplier W[k+1, K]
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = t + q * kGjThreads;
        Ds[e >> 6][e & (kNB - 1)] = xv[q];
      }
      stash_b(pv);
      __syncthreads();  // X has been read
      if (t == 0) {
        __hip_atomic_fetch_add(a.lflag + k, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = dseen >= 1 || flow_wait(a.dflag + k, 1, a.bits);
      }
      if (!finish_wait(ok)) continue;
      stash_dinv(a.dinv + (int64_t)k * kNB * kNB);
      __syncthreads();
      double acc[16];
      product(acc);  // R
      store_out(acc, k0, k2, k0 + kNB, k2, ncols);
      flow_signal(a.pdone + k * a.S + k + 2);  // every wave is past the product
      if (t == 0) __hip_atomic_fetch_add(tile_cnt(a, k, k + 2), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // Bs[j][k] = R(k, j); As[i][k] = W[K, k+2](k, i): the multiplier W[k+2, K]
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = jr + x * 16 + (lane >> 4) + 4 * q, i = ic + y * 16 + lr;
            Bs[j][i] = acc[(x * 2 + y) * 4 + q];
          }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = t + q * kGjThreads;
        As[e >> 6][e & (kNB - 1)] = pv[q];
      }
      __syncthreads();
      product(acc);  // W[k+2, K] R
#pragma unroll
      for (int q = 0; q < 16; ++q) c2[q] -= acc[q];
      product_a(acc, Ds);  // W[k+1, K] R
#pragma unroll
      for (int q = 0; q < 16; ++q) c1[q] -= acc[q];
      store_out(c1, k1, k2, n, k2, ncols);
      store_out(c2, k2, k2, n, k2, ncols);
      wait_stores();
      __syncthreads();
      if (t == 0) {
        __hip_atomic_fetch_add(tile_cnt(a, k + 1, k + 2), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(tile_cnt(a, k + 2, k + 2), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(a.cnt + k * a.S + k + 2, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      continue;
    }
    if (u < f.nP) {
      // ---- P(k, j): R_j = D_k^{-1} W[K, j]
      const int j = pc ? (u == 1 ? k + 1 : f.j0 + u) : f.j0 + u;
      const int64_t cj = (int64_t)j * kNB;
      bool ok = true;
      if (t == 0) {
        ok = flow_wait(a.dflag + k, 1, a.bits);
        if (ok && k >= 1) ok = flow_wait(tile_cnt(a, k, j), tile_need(k, j, k), a.bits);
        if (ok && f.hasL && j == k + 1) ok = flow_wait(a.lflag + k, pc ? 2 : 1, a.bits);
      }
      if (!finish_wait(ok)) continue;
      double xv[16];
      load_tile(xv, k0, cj, k0 + f.nb, f.c0, ncols);
      stash_dinv(a.dinv + (int64_t)k * kNB * kNB);
      stash_b(xv);
      __syncthreads();
      double acc[16];
      product(acc);
      store_out(acc, k0, cj, k0 + f.nb, f.c0, ncols);
      flow_signal(a.pdone + k * a.S + j);
      if (t == 0) {
        __hip_atomic_fetch_add(tile_cnt(a, k, j), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(a.cnt + k * a.S + j, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (a.ex.bt && k == R - 1) store_bt(acc, k0, cj);
      continue;
    }
    u -= f.nP;
    // ---- U(k, i, j): W[i, j] -= W[i, K] R_j
    // (rows in each strip from the one below the pivot down, then from the top:
    // the tiles the next pivot steps read first)
    int i, j;
    if (f.hasL) {
      if (u < R - 2) {
        j = k + 1;
        i = (k + 2 + u) % R;
      } else {
        u -= R - 2;
        j = k + 2 + u / (R - 1);
        i = (k + 1 + u % (R - 1)) % R;
      }
    } else {
      j = f.j0 + u / (R - 1);
      i = (k + 1 + u % (R - 1)) % R;
    }
    if (pc && j == k + 2 && (i == k + 1 || i == k + 2)) continue;  // formed by PC(k)
    const int64_t ri = (int64_t)i * kNB, cj = (int64_t)j * kNB;
    bool ok = true;
    if (t == 0) {
      ok = flow_wait(a.pdone + k * a.S + j, 1, a.bits);
      if (ok && k >= 1) ok = flow_wait(tile_cnt(a, i, k), k, a.bits) && flow_wait(tile_cnt(a, i, j), tile_need(i, j, k), a.bits);
      if (ok && i == k - 1) ok = flow_wait(a.cnt + (k - 1) * a.S + j, flow_target(a, k - 1, j), a.bits);
    }
    if (!finish_wait(ok)) continue;
    double mv[16], rv[16], cv[16];
    load_tile(mv, ri, k0, n, k0, k0 + f.nb);
    load_tile(rv, k0, cj, k0 + f.nb, f.c0, ncols);
    load_out(cv, ri, cj, n, f.c0, ncols);
    stash_a(mv);
    stash_b(rv);
    __syncthreads();
    double acc[16];
    product(acc);
#pragma unroll
    for (int q = 0; q < 16; ++q) cv[q] -= acc[q];
    store_out(cv, ri, cj, n, f.c0, ncols);
    flow_signal(tile_cnt(a, i, j));
    if (t == 0) __hip_atomic_fetch_add(a.cnt + k * a.S + j, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a.ex.bt && k == R - 1) store_bt(cv, ri, cj);
  }
}

// D_0 = W[0:nb, 0:nb] inverted into dinv block 0 (as k_gj_inv0), and the
// flow counters cleared, before the dataflow launch.
__global__ __launch_bounds__(kGjThreads) void k_gj_flow_init(GjFlow a) {
  __shared__ double Ds[kNB][kLds];
  __shared__ double Es[kNB][kLds];
  __shared__ InvBlk inv;
  __shared__ double rsum[kGjThreads / kWave];
  const int t = threadIdx.x;
  // the first pivot block's loads go out first (columns 0..63: untouched by
  // the right-hand-side column written below)
  const int nb = (int)(a.n < kNB ? a.n : kNB);
  double dv[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + q * kGjThreads, r = e & (kNB - 1), c = e >> 6;
    dv[q] = (r < nb && c < nb) ? a.W[r + (int64_t)c * a.ldw] : (r == c ? 1.0 : 0.0);
  }
  // every other load goes out before any store: the one-launch form has
  // n <= kFlowMaxRows * 64, so each thread's entries are one batch
  constexpr int kPer = kFlowMaxRows * kNB / kGjThreads;
  double g1[kPer], g2[kPer], d1[kPer], d2[kPer], xr[kPer];
  if (a.pre.g) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int64_t j = t + (int64_t)u * kGjThreads;
      const bool in = j < a.n;
      g1[u] = in ? a.pre.g[j] : 0.0;
      g2[u] = in ? a.pre.g2[j] : 0.0;
      d1[u] = in ? a.W[j + j * a.ldw] : 0.0;
      d2[u] = in ? a.W[j + (a.n + j) * a.ldw] : 0.0;
    }
  }
  if (a.ex.reset && a.ex.reset_xr) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int64_t j = t + (int64_t)u * kGjThreads;
      xr[u] = j < a.n ? a.ex.reset_xr[j] : 0.0;
    }
  }
  const int64_t nint = 3 * (int64_t)a.R * a.S + 2 * a.R + 1;  // tcnt, cnt, pdone, dflag, lflag, ticket
  for (int64_t e = t; e < nint; e += kGjThreads) a.tcnt[e] = 0;
  if (a.ex.reset) {
    // the loop state cleared (its bits included) before anything below can
    // raise a bit, and ||x_ref||^2 for the relative error
    constexpr int kWords = (int)(sizeof(LoopState) / sizeof(int));
    int* lw = (int*)a.ex.reset;
    for (int e = t; e < kWords; e += kGjThreads) lw[e] = 0;
    if (a.ex.reset_xr) {
      double sq = 0.0;
#pragma unroll
      for (int u = 0; u < kPer; ++u) sq += xr[u] * xr[u];
      sq = block_sum<kGjThreads>(sq, rsum);  // its barrier also orders the zeroing before the store
      if (t == 0) a.ex.reset->scal[1] = sq;
    }
    __syncthreads();
  }
  if (a.pre.g) {
    // the right-hand-side column g = g1 - g2 and the screen of g and of the
    // diagonals of the two Gram blocks (columns 0..n-1 and n..2n-1 of W)
    int bad = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int64_t j = t + (int64_t)u * kGjThreads;
      if (j < a.n) {
        const double v = g1[u] - g2[u];
        a.pre.g[j] = v;
        a.pre.gcol[j] = v;
        bad |= !isfinite(v) || !isfinite(d1[u]) || !isfinite(d2[u]);
      }
    }
    if (__syncthreads_or(bad)) {
      if (t == 0) atomicOr(a.bits, kBitNonfinite);
      return;
    }
  }
  if (__hip_atomic_load(a.bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + q * kGjThreads;
    Ds[e & (kNB - 1)][e >> 6] = dv[q];
  }
  __syncthreads();
  if (!invert64_blk(&Ds[0][0], &Es[0][0], inv)) {
    if (t == 0) atomicOr(a.bits, kBitNotSpd);
    return;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + q * kGjThreads;
    a.dinv[e] = Ds[e >> 6][e & (kNB - 1)];
  }
  __syncthreads();
  if (t == 0) a.dflag[0] = 1;
}

static bool flow_fits(int64_t n) { return (n + kNB - 1) / kNB <= kFlowMaxRows; }
bool gj_one_launch(int64_t n, int64_t nrhs) { return flow_fits(n) && nrhs > 0; }

size_t gj_scratch_bytes(int64_t n, int64_t ncols) {
  size_t b = sizeof(double) * 2 * kNB * kNB;  // the step-by-step form
  if (flow_fits(n)) {
    const int64_t R = (n + kNB - 1) / kNB, S = (ncols + kNB - 1) / kNB;
    const size_t f = sizeof(double) * R * kNB * kNB + sizeof(int) * (3 * R * S + 2 * R + 1);
    if (f > b) b = f;
  }
  return b;
}


void launch_gj(hipStream_t s, int64_t n, int64_t nrhs, double* W, int64_t ldw, void* scratch, int* bits,
               const GjCombine* pre, const GjExtras* ex) {
  const int64_t ncols = n + nrhs;
  const int row_tiles = (int)((n + kNB - 1) / kNB);
  if (gj_one_launch(n, nrhs)) {
    GjFlow a;
    a.W = W;
    a.ldw = ldw;
    a.n = n;
    a.ncols = ncols;
    a.R = row_tiles;
    a.S = (int)((ncols + kNB - 1) / kNB);
    a.dinv = (double*)scratch;
    a.tcnt = (int*)(a.dinv + (int64_t)a.R * kNB * kNB);
    a.cnt = a.tcnt + a.R * a.S;
    a.pdone = a.cnt + a.R * a.S;
    a.dflag = a.pdone + a.R * a.S;
    a.lflag = a.dflag + a.R;
    a.ticket = (unsigned*)(a.lflag + a.R);
    a.bits = bits;
    a.pre = pre ? *pre : GjCombine{nullptr, nullptr, nullptr};
    a.ex = ex ? *ex : GjExtras{nullptr, nullptr, nullptr, 0, 0, 0};
    hipLaunchKernelGGL(k_gj_flow_init, dim3(1), dim3(kGjThreads), 0, s, a);
    hipLaunchKernelGGL(k_gj_flow, dim3(kFlowWgs), dim3(kGjThreads), 0, s, a);
    return;
  }
  if (pre) launch_border_combine(s, n, pre->g, pre->g2, W, W + n * ldw, ldw, pre->gcol, bits);
  double* dinv = (double*)scratch;
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
