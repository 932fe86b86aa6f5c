// k_rkblock.hip -- SP-RK-RGS inner steps (Alg. 2 steps 8-11) in blocks of
// kRB steps spread over the whole GPU.
//
// The column draws do not depend on the iterate, so the kRB steps of a block
// are known in advance: u_t = A1_(j1(t)), v_t = A1_(j2(t)).  With the
// incremental state s = w - A1 z, the block's scalars follow from inner
// products only:
//   gamma_t = (bhat_{j1(t)} - u_t^T w_0 - sum_{tau<t} gamma_tau u_t^T u_tau) / c_{j1(t)}
//   delta_t = (v_t^T s_0 + sum_{tau<=t} gamma_tau v_t^T u_tau
//              - sum_{tau<t} delta_tau v_t^T v_tau) / c_{j2(t)}
// after which w += sum gamma_t u_t, s += sum gamma_t u_t - sum delta_t v_t and
// z_{j2(t)} += delta_t -- the same iterates as kRB single steps in exact
// arithmetic.  A block is two launches:
//   k_rkb_step    per row slice (all CUs): w and s of the slice take the
//                 previous block's update, then the slice's partial block of
//                 C = [U V]^T [U V w_0 s_0] on the matrix cores;
//   k_rkb_close   the slices added in slice order (deterministic); the last
//                 workgroup to finish runs the 2 kRB scalar recurrences and the
//                 z updates in one wave.
// One more k_rkb_step without a next block applies the last block's update.
#include "ils_common.hpp"
#include "k_rand.hpp"

namespace ils {

constexpr int kRB = 32;              // steps per block
constexpr int kRBX = 2 * kRB;        // gathered columns u_0.., v_0..
constexpr int kRBY = kRBX + 16;      // + w_0, s_0 and zero padding
constexpr int kRBS = 128;            // rows of a slice held in LDS at once
constexpr int kRBL = kRBS + 1;       // LDS row stride

template <typename T>
struct RbMma;
template <>
struct RbMma<double> {
  typedef v4d acc_t;
  __device__ static acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct RbMma<float> {
  typedef v4f acc_t;
  __device__ static acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

__device__ inline bool rb_skip(const int* inner_done, const int* outer_done) {
  return *(volatile const int*)inner_done || *(volatile const int*)outer_done;
}

// Column c of a block's gathered set [U V] (nullptr past the block's end).
template <typename T>
__device__ inline const T* rb_col(const T* A1, int64_t lda, const int* j1, const int* j2, int bt, int c) {
  if (c < kRB) return c < bt ? A1 + (int64_t)j1[c] * lda : nullptr;
  return c - kRB < bt ? A1 + (int64_t)j2[c - kRB] * lda : nullptr;
}

// Workgroup = one slice of rows, visited in chunks of kRBS rows.  Thread
// (lk, cg) = (t % 16, t / 16) loads rows lk, lk + 16, ... of gathered columns
// cg, cg + 16, cg + 32, cg + 48; the loads of both blocks are issued together.
// Previous block (pbt > 0): row i of the chunk forms dw = sum gamma_t u_t(i)
// (thread i) and dv = sum delta_t v_t(i) (thread 128 + i), each as two chains
// of 16 in column order, and w(i) += dw, s(i) += dw - dv.  This block (bt > 0):
// wave g accumulates rows 16g..16g+15 of C against all kRBY columns (the u
// rows skip the v columns, which the recurrences never read).
template <typename T>
__global__ __launch_bounds__(256) void k_rkb_step(const T* __restrict__ A1, int64_t lda, int64_t p,
                                                  const int* __restrict__ pj1, const int* __restrict__ pj2, int pbt,
                                                  const double* __restrict__ coef, const int* __restrict__ j1,
                                                  const int* __restrict__ j2, int bt, T* __restrict__ w,
                                                  T* __restrict__ s, int64_t slice_rows, T* __restrict__ part,
                                                  const int* inner_done, const int* outer_done) {
  if (rb_skip(inner_done, outer_done)) return;
  typedef typename RbMma<T>::acc_t acc_t;
  __shared__ T Ms[kRBY][kRBL];
  __shared__ double cf[kRBX];
  __shared__ double dvs[kRBS];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, lr = lane & 15;
  const int lk = t & 15, cg = t >> 4;
  const T* ps[4];
  const T* ns[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ps[q] = rb_col(A1, lda, pj1, pj2, pbt, cg + 16 * q);
    ns[q] = rb_col(A1, lda, j1, j2, bt, cg + 16 * q);
  }
  if (t < kRBX) cf[t] = pbt > 0 ? coef[t] : 0.0;
  for (int e = t; e < (kRBY - kRBX - 2) * kRBL; e += 256) Ms[kRBX + 2 + e / kRBL][e % kRBL] = (T)0;
  acc_t acc[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) acc[c] = acc_t{};
  const int64_t s0 = (int64_t)blockIdx.x * slice_rows;
  const int64_t s1 = s0 + slice_rows < p ? s0 + slice_rows : p;
  for (int64_t r0 = s0; r0 < s1; r0 += kRBS) {
    const int nr = (int)(s1 - r0 < kRBS ? s1 - r0 : kRBS);
    const int nr16 = (nr + 15) & ~15;
    T pv[4][kRBS / 16], nv[4][kRBS / 16];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int rr = 0; rr < kRBS / 16; ++rr) {
        const int k = lk + 16 * rr;
        pv[q][rr] = (ps[q] && k < nr) ? ps[q][r0 + k] : (T)0;
        nv[q][rr] = (ns[q] && k < nr) ? ns[q][r0 + k] : (T)0;
      }
    const int i = t & (kRBS - 1);
    T wi = (T)0, si = (T)0;
    if (i < nr) {
      wi = w[r0 + i];
      si = s[r0 + i];
    }
    __syncthreads();  // the previous chunk's matrix-core reads of Ms are done
    if (pbt > 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int rr = 0; rr < kRBS / 16; ++rr) Ms[cg + 16 * q][lk + 16 * rr] = pv[q][rr];
      __syncthreads();
      const int c0 = t < kRBS ? 0 : kRB;  // gamma (u) or delta (v) half
      double h0 = 0.0, h1 = 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) h0 = fma(cf[c0 + u], (double)Ms[c0 + u][i], h0);
#pragma unroll
      for (int u = 16; u < 32; ++u) h1 = fma(cf[c0 + u], (double)Ms[c0 + u][i], h1);
      if (t >= kRBS) dvs[i] = h0 + h1;
      __syncthreads();
      if (t < kRBS && i < nr) {
        const double dw = h0 + h1;
        wi = (T)((double)wi + dw);
        si = (T)((double)si + (dw - dvs[i]));
        w[r0 + i] = wi;
        s[r0 + i] = si;
      }
      __syncthreads();  // the update's reads of Ms are done
    }
    if (bt == 0) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int rr = 0; rr < kRBS / 16; ++rr) Ms[cg + 16 * q][lk + 16 * rr] = nv[q][rr];
    if (t < kRBS) {
      Ms[kRBX][i] = wi;
      Ms[kRBX + 1][i] = si;
    }
    __syncthreads();
    for (int kk = 0; kk < nr16; kk += 4) {
      const int kr = kk + (lane >> 4);
      const T a = Ms[16 * wv + lr][kr];
#pragma unroll
      for (int c = 0; c < 5; ++c)
        if (wv >= 2 || c < 2 || c == 4) acc[c] = RbMma<T>::run(a, Ms[16 * c + lr][kr], acc[c]);
    }
  }
  if (bt == 0) return;
  T* P = part + (int64_t)blockIdx.x * (kRBX * kRBY);
#pragma unroll
  for (int c = 0; c < 5; ++c)
    if (wv >= 2 || c < 2 || c == 4)
#pragma unroll
      for (int v = 0; v < 4; ++v) P[(16 * wv + RbMma<T>::row(lane, v)) * kRBY + 16 * c + lr] = acc[c][v];
}

// Broadcast lane `src`'s value to the whole wave (32-bit lane reads).
__device__ inline double lane_value(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

__device__ inline double rb_load(const double* C, int e) {
  return __hip_atomic_load(C + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The block's scalar recurrences are two lower-triangular solves of size bt:
//   c_{j1(t)} gamma_t + sum_{tau<t} (u_t^T u_tau) gamma_tau = bhat_{j1(t)} - u_t^T w_0
//   c_{j2(t)} delta_t + sum_{tau<t} (v_t^T v_tau) delta_tau
//                     = v_t^T s_0 + sum_{tau<=t} (v_t^T u_tau) gamma_tau.
// One wave: lane tau keeps its row of both systems in registers; step t takes
// lane t's unknown, broadcasts it (lane reads) and every lane subtracts its
// term (column-oriented substitution, no reductions).  z_b then takes, for
// each distinct column b of the block, the sum of its delta_t in step order.
__device__ __attribute__((always_inline)) inline void rkb_recur_wave(const double* C, int bt, const int* __restrict__ j1, const int* __restrict__ j2,
                               const double* __restrict__ tgt, const double* __restrict__ cn,
                               double* __restrict__ z, double* __restrict__ coef) {
  const int lane = threadIdx.x & 63;
  const int tau = lane < kRB ? lane : kRB - 1;  // lanes >= kRB mirror the last row, unused
  const bool live = lane < bt;
  const int a = live ? j1[lane] : 0, b = live ? j2[lane] : -1;
  const double rcg = live ? 1.0 / cn[a] : 0.0;
  const double rcd = live ? 1.0 / cn[b] : 0.0;
  double rg = live ? tgt[a] - rb_load(C, tau * kRBY + kRBX) : 0.0;   // gamma system right-hand side
  double rd = live ? rb_load(C, (kRB + tau) * kRBY + kRBX + 1) : 0.0;  // delta system right-hand side
  double uu[kRB], vu[kRB], vv[kRB];
#pragma unroll
  for (int k = 0; k < kRB; ++k) {
    uu[k] = rb_load(C, tau * kRBY + k);
    vu[k] = rb_load(C, (kRB + tau) * kRBY + k);
    vv[k] = rb_load(C, (kRB + tau) * kRBY + kRB + k);
  }
  double gam = 0.0, del = 0.0;
#pragma unroll
  for (int t = 0; t < kRB; ++t) {
    if (t < bt) {
      const double g = lane_value(rg * rcg, t);
      if (lane == t) gam = g;
      if (lane > t) rg = fma(-uu[t], g, rg);
      if (lane >= t) rd = fma(vu[t], g, rd);
    }
  }
#pragma unroll
  for (int t = 0; t < kRB; ++t) {
    if (t < bt) {
      const double d = lane_value(rd * rcd, t);
      if (lane == t) del = d;
      if (lane > t) rd = fma(-vv[t], d, rd);
    }
  }
  if (lane < kRB) {
    coef[lane] = live ? gam : 0.0;
    coef[kRB + lane] = live ? del : 0.0;
  }
  bool first = live;
  double sum = 0.0;
  for (int u = 0; u < bt; ++u) {
    const int bu = __builtin_amdgcn_readlane(b, u);
    const double du = lane_value(del, u);
    if (bu == b) {
      if (u < lane) first = false;
      else sum += du;
    }
  }
  if (first) z[b] += sum;
}

// C[i][j] = sum over slices of the partial blocks.  Workgroup = 32 entries
// x 8 slice groups: group g adds slices g, g + 8, ... (up to 32 loads in
// flight per thread), then the eight group sums are added in group order
// (deterministic).  Entries the recurrences never read (u rows against v
// columns) are left out.  The last workgroup to arrive runs the recurrences.
constexpr int kRedE = 32;       // entries per workgroup
constexpr int kRedG = 8;        // slice groups per workgroup
constexpr int kRedDepth = 32;   // loads in flight per thread

__device__ inline bool rb_needed(int e) {
  const int r = e / kRBY, c = e % kRBY;
  return !(r < kRB && c >= kRB && c < kRBX);
}

template <typename T>
__global__ __launch_bounds__(256) void k_rkb_close(const T* __restrict__ part, int nslices, double* __restrict__ C,
                                                   unsigned* arrive, int bt, const int* __restrict__ j1,
                                                   const int* __restrict__ j2, const double* __restrict__ tgt,
                                                   const double* __restrict__ cn, double* __restrict__ z,
                                                   double* __restrict__ coef, const int* inner_done,
                                                   const int* outer_done) {
  if (rb_skip(inner_done, outer_done)) return;
  __shared__ double red[kRedG][kRedE];
  __shared__ int is_last;
  const int lane = threadIdx.x & 63;
  const int le = threadIdx.x & (kRedE - 1), g = threadIdx.x / kRedE;
  const int e = blockIdx.x * kRedE + le;
  double acc = 0.0;
  if (e < kRBX * kRBY && rb_needed(e)) {
    for (int s0 = g; s0 < nslices; s0 += kRedG * kRedDepth) {
      T v[kRedDepth];
#pragma unroll
      for (int u = 0; u < kRedDepth; ++u) {
        const int sl = s0 + kRedG * u;
        v[u] = sl < nslices ? part[(int64_t)sl * (kRBX * kRBY) + e] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < kRedDepth; ++u) acc += (double)v[u];
    }
  }
  red[g][le] = acc;
  __syncthreads();
  // C is handed to the last workgroup through device-scope stores and loads
  // (past the per-XCD caches): the writing wave waits until its stores are
  // acknowledged and then counts, so no cache write-back or invalidation
  // (a device-scope fence in every workgroup) is needed
  if (threadIdx.x < kRedE && e < kRBX * kRBY) {
    double tot = red[0][le];
#pragma unroll
    for (int u = 1; u < kRedG; ++u) tot += red[u][le];
    __hip_atomic_store(C + e, tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __asm__ __volatile__("" ::: "memory");
  if (threadIdx.x == 0) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): wave 0's stores of C have completed
    is_last = __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last) return;
  if (threadIdx.x >= 64) return;
  rkb_recur_wave(C, bt, j1, j2, tgt, cn, z, coef);
  if (lane == 0) *arrive = 0;
}

int64_t rk_block_steps() { return kRB; }

size_t rk_block_scratch(int64_t p) {
  // partial blocks of every slice (as doubles) plus C and the coefficients
  const int64_t rows = rk_block_slice_rows(p);
  const int64_t nsl = (p + rows - 1) / rows;
  return (size_t)nsl * kRBX * kRBY + (size_t)kRBX * kRBY + kRBX;
}

int64_t rk_block_slice_rows(int64_t p) {
  int64_t rows = (p + 255) / 256;  // about one slice per CU
  rows = (rows + 15) / 16 * 16;
  return rows < 16 ? 16 : rows;
}

template <typename T>
static void rkb_run(hipStream_t st, const T* A1, int64_t lda, int64_t p, const double* tgt, const double* cn,
                    const int* j1, const int* j2, int64_t count, T* w, T* s, double* z, double* scratch,
                    unsigned* arrive, const int* inner_done, const int* outer_done) {
  if (count <= 0) return;
  const int64_t rows = rk_block_slice_rows(p);
  const int nsl = (int)((p + rows - 1) / rows);
  T* part = (T*)scratch;
  double* C = scratch + (int64_t)nsl * kRBX * kRBY;
  double* coef = C + kRBX * kRBY;
  int pbt = 0;
  int64_t pt0 = 0;
  for (int64_t t0 = 0;; t0 += kRB) {
    const int64_t left = count - t0 > 0 ? count - t0 : 0;
    const int bt = (int)(left < kRB ? left : kRB);  // 0: only the last block's update
    if (bt == 0 && pbt == 0) break;
    hipLaunchKernelGGL((k_rkb_step<T>), dim3((unsigned)nsl), dim3(256), 0, st, A1, lda, p, j1 + pt0, j2 + pt0, pbt,
                       (const double*)coef, j1 + t0, j2 + t0, bt, w, s, rows, part, inner_done, outer_done);
    if (bt == 0) break;
    hipLaunchKernelGGL((k_rkb_close<T>), dim3((kRBX * kRBY + kRedE - 1) / kRedE), dim3(256), 0, st, (const T*)part, nsl, C,
                       arrive, bt, j1 + t0, j2 + t0, tgt, cn, z, coef, inner_done, outer_done);
    pbt = bt;
    pt0 = t0;
  }
}

void launch_rk_blocks(hipStream_t st, const double* A1, int64_t lda, int64_t p, const double* tgt, const double* cn,
                      const int* j1, const int* j2, int64_t count, double* w, double* s, double* z, double* scratch,
                      unsigned* arrive, const int* inner_done, const int* outer_done) {
  rkb_run<double>(st, A1, lda, p, tgt, cn, j1, j2, count, w, s, z, scratch, arrive, inner_done, outer_done);
}

void launch_rk_blocks_f32(hipStream_t st, const float* A1, int64_t lda, int64_t p, const double* tgt,
                          const double* cn, const int* j1, const int* j2, int64_t count, float* w, float* s,
                          double* z, double* scratch, unsigned* arrive, const int* inner_done,
                          const int* outer_done) {
  rkb_run<float>(st, A1, lda, p, tgt, cn, j1, j2, count, w, s, z, scratch, arrive, inner_done, outer_done);
}

}  // namespace ils
