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

// ------------------------------------------------- 64 x 64 SPD inverse by 16 x 16 blocks
// In-place Gauss-Jordan inversion carried out on 4 x 4 blocks of 16 x 16:
// for each block pivot K with P = A_KK^{-1},
//   A_KJ <- P A_KJ,  A_IK <- -A_IK P,  A_IJ <- A_IJ + A_IK(new) A_KJ(old),
//   A_KK <- P          (I, J != K),
// with the block products on the FP64 matrix cores and the 16 x 16 inversions
// done by one wave in registers.  Two LDS buffers alternate as the matrix
// before and after each block step.  Wave 0 forms the next diagonal block
// and inverts it while the other three waves update the rest, so one block
// step costs about one 16 x 16 inversion.
constexpr int kLds = kNB + 1;  // row stride (doubles) of the 64 x 64 LDS buffers

struct InvBlk {
  double x[16][17];  // wave 0's 16 x 16 staging block
  int bad;
};

__device__ inline double lane_read(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Lane K of each row of 16 lanes, for every lane (DPP row broadcast; on a
// double this is one 64-bit DPP move, which makes the 16 x 16 inversion below
// about 9 % faster than two 32-bit moves).
template <int K>
__device__ inline double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 | K, 0xF, 0xF, true);
}

// 1/x to full double precision from the hardware estimate r0:
// r0 (1 + e + e^2) with e = 1 - x r0 (the estimate's error cubed is far
// below double rounding).
__device__ inline double recip_e2(double x) {
  const double r0 = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r0, 1.0);
  return fma(r0, fma(e, e, e), r0);
}

// One pivot of leaf_inv16.  The pivot row is left unscaled: every other row
// takes row_i - (a_ik / a_kk) row_k, column k takes -a_ik / a_kk on those
// rows and 1 on row k, and row k's pivot a_kk is kept in dsv by the lanes of
// row k.  The inverse is the result with each row divided by its pivot.
template <int K>
__device__ inline void leaf_pivot(double (&a)[4], int lane, bool& bad, double& dsv) {
  constexpr int kg = K >> 2, kc = K & 3;
  const int i = lane & 15, g = lane >> 4;
  double pr[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) pr[c] = row_bcast<K>(a[c]);
  const double pc = __shfl(a[kc], i | (kg << 4));
  const double piv = lane_read(a[kc], K | (kg << 4));
  bad |= !(piv > 0.0);
  const double r = recip_e2(piv);
  const bool prow = i == K;
  const double beta = prow ? 0.0 : -pc * r;
  dsv = prow ? piv : dsv;
#pragma unroll
  for (int c = 0; c < 4; ++c) a[c] = fma(beta, pr[c], a[c]);
  if (g == kg) a[kc] = prow ? 1.0 : beta;
  if constexpr (K < 15) leaf_pivot<K + 1>(a, lane, bad, dsv);
}

// In-place inverse of a 16 x 16 SPD block by one wave: lane l holds row l % 16,
// columns 4 (l / 16) .. 4 (l / 16) + 3.  Pivot k broadcasts row k within each
// group of 16 lanes (DPP) and the column-k entry of each row across the
// groups (lane permute).  Returns false when a pivot is not > 0.
__device__ inline bool leaf_inv16(double (&a)[4], int lane) {
  bool bad = false;
  double dsv = 1.0;
  leaf_pivot<0>(a, lane, bad, dsv);
  const double rd = recip(dsv);
#pragma unroll
  for (int c = 0; c < 4; ++c) a[c] *= rd;
  return !bad;
}

__device__ inline const double* blk16(const double* B, int I, int J) { return B + 16 * I * kLds + 16 * J; }
__device__ inline double* blk16(double* B, int I, int J) { return B + 16 * I * kLds + 16 * J; }

// acc += X Y for 16 x 16 blocks in LDS (row strides ldx, ldy), one wave.
// Lane l supplies X[l % 16][k + l / 16] and Y[k + l / 16][l % 16]; acc[v] is
// entry (l / 16 + 4 v, l % 16).
__device__ inline v4d mm16(const double* X, int ldx, const double* Y, int ldy, v4d acc, int lane) {
  const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 16; kk += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[lr * ldx + kk + lq], Y[(kk + lq) * ldy + lr], acc, 0, 0, 0);
  return acc;
}
__device__ inline v4d ld16(const double* Z, int ldz, int lane) {
  const int lr = lane & 15, lq = lane >> 4;
  return v4d{Z[lq * ldz + lr], Z[(lq + 4) * ldz + lr], Z[(lq + 8) * ldz + lr], Z[(lq + 12) * ldz + lr]};
}
__device__ inline void st16(double* Z, int ldz, v4d v, int lane) {
  const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
  for (int e = 0; e < 4; ++e) Z[(lq + 4 * e) * ldz + lr] = v[e];
}

// Row I != K of a block step: nxt_IK = -cur_IK P, then
// nxt_IJ = cur_IJ + nxt_IK cur_KJ for J != K, J != skip.
__device__ inline void blk_row(const double* cur, double* nxt, const double* P, int I, int K, int skip, int lane) {
  const v4d zero = {0.0, 0.0, 0.0, 0.0};
  const v4d x = mm16(blk16(cur, I, K), kLds, P, kLds, zero, lane);
  st16(blk16(nxt, I, K), kLds, -x, lane);
  __threadfence_block();
#pragma unroll
  for (int J = 0; J < 4; ++J) {
    if (J == K || J == skip) continue;
    const v4d acc = mm16(blk16(nxt, I, K), kLds, blk16(cur, K, J), kLds, ld16(blk16(cur, I, J), kLds, lane), lane);
    st16(blk16(nxt, I, J), kLds, acc, lane);
  }
}

// Inverse of the 64 x 64 SPD matrix in B0 (row stride kLds, LDS), written back
// into B0; B1 is a second buffer of the same shape.  All 256 threads call it
// after a barrier that makes B0 complete; returns false in every thread when
// a pivot is not > 0 (the matrix is not positive definite).
// The block steps of invert64_blk, given the inverse of B0's (0,0) block
// already in B1's (0,0) block and S.bad set (a caller that forms B0 itself can
// invert that first block while the rest is still being formed).
__device__ __attribute__((always_inline)) inline bool invert64_steps(double* B0, double* B1, InvBlk& S) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const v4d zero = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int K = 0; K < 4; ++K) {
    double* cur = (K & 1) ? B1 : B0;
    double* nxt = (K & 1) ? B0 : B1;
    const double* P = blk16(nxt, K, K);
    if (K < 3) {
      const int Ia = K == 0 ? 2 : 0, Ib = K == 2 ? 1 : 3;  // the rows other than K, K + 1
      if (w == 0) {
        // next diagonal block cur_(K+1)(K+1) - cur_(K+1)K P cur_K(K+1), inverted
        // into cur_(K+1)(K+1), which no other wave reads in this step
        const v4d x = mm16(blk16(cur, K + 1, K), kLds, P, kLds, zero, lane);
        st16(&S.x[0][0], 17, -x, lane);
        __threadfence_block();
        const v4d d = mm16(&S.x[0][0], 17, blk16(cur, K, K + 1), kLds, ld16(blk16(cur, K + 1, K + 1), kLds, lane),
                           lane);
        __threadfence_block();
        st16(&S.x[0][0], 17, d, lane);
        __threadfence_block();
        double a[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) a[c] = S.x[li][4 * lg + c];
        const bool ok = leaf_inv16(a, lane);
        double* D = blk16(cur, K + 1, K + 1);
#pragma unroll
        for (int c = 0; c < 4; ++c) D[li * kLds + 4 * lg + c] = a[c];
        if (!ok && lane == 0) S.bad = 1;
      } else if (w == 1) {
        blk_row(cur, nxt, P, Ia, K, -1, lane);
      } else if (w == 2) {
        blk_row(cur, nxt, P, Ib, K, -1, lane);
      } else {
#pragma unroll
        for (int J = 0; J < 4; ++J)
          if (J != K) st16(blk16(nxt, K, J), kLds, mm16(P, kLds, blk16(cur, K, J), kLds, zero, lane), lane);
        blk_row(cur, nxt, P, K + 1, K, K + 1, lane);  // row K + 1 without its diagonal block
      }
    } else if (w < 3) {
      blk_row(cur, nxt, P, w, K, -1, lane);
    } else {
#pragma unroll
      for (int J = 0; J < 4; ++J)
        if (J != K) st16(blk16(nxt, K, J), kLds, mm16(P, kLds, blk16(cur, K, J), kLds, zero, lane), lane);
    }
    __syncthreads();
  }
  return S.bad == 0;
}

__device__ __attribute__((always_inline)) inline bool invert64_blk(double* B0, double* B1, InvBlk& S) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  if (w == 0) {
    double a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = B0[li * kLds + 4 * lg + c];
    const bool ok = leaf_inv16(a, lane);
#pragma unroll
    for (int c = 0; c < 4; ++c) B1[li * kLds + 4 * lg + c] = a[c];
    if (lane == 0) S.bad = ok ? 0 : 1;
  }
  __syncthreads();
  return invert64_steps(B0, B1, S);
}

}  // namespace ils
