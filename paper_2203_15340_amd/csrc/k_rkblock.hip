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
// arithmetic.  A block is four launches:
//   k_rkb_gram   C = [U V]^T [U V w_0 s_0] on the matrix cores, split over row
//                slices (all CUs), partial blocks per slice;
//   k_rkb_reduce the slices added in slice order (deterministic);
//   k_rkb_recur  one wave: the 2 kRB scalar recurrences and the z updates;
//   k_rkb_update w and s for all p rows.
#include "ils_common.hpp"
#include "k_rand.hpp"

namespace ils {

constexpr int kRB = 32;              // steps per block
constexpr int kRBX = 2 * kRB;        // gathered columns u_0.., v_0..
constexpr int kRBY = kRBX + 16;      // + w_0, s_0 and zero padding

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

// Workgroup = one slice of at most kRBS rows; wave w forms output rows
// 16w..16w+15 (of the kRBX gathered columns) against all kRBY columns.  The
// whole slice is loaded at once (up to forty loads in flight per thread),
// staged in LDS, and then consumed by the matrix cores.
constexpr int kRBS = 128;  // rows per slice at most

template <typename T>
__global__ __launch_bounds__(256) void k_rkb_gram(const T* __restrict__ A1, int64_t lda, int64_t p,
                                                  const int* __restrict__ j1, const int* __restrict__ j2, int bt,
                                                  const T* __restrict__ w, const T* __restrict__ s,
                                                  int64_t slice_rows, T* __restrict__ part, const int* inner_done,
                                                  const int* outer_done) {
  if (rb_skip(inner_done, outer_done)) return;
  typedef typename RbMma<T>::acc_t acc_t;
  __shared__ T Ms[kRBY][kRBS + 1];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, lr = lane & 15;
  const int lk = t & 15, cg = t >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * slice_rows;
  const int64_t r1 = r0 + slice_rows < p ? r0 + slice_rows : p;
  const int nr = (int)(r1 - r0);
  const int nr16 = (nr + 15) & ~15;
  // the (up to) five gathered columns this thread loads: c = cg + 16 q
  const T* src[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const int c = cg + 16 * q;
    const T* ptr = nullptr;
    if (c < kRB) {
      if (c < bt) ptr = A1 + (int64_t)j1[c] * lda;
    } else if (c < kRBX) {
      if (c - kRB < bt) ptr = A1 + (int64_t)j2[c - kRB] * lda;
    } else if (c == kRBX) {
      ptr = w;
    } else if (c == kRBX + 1) {
      ptr = s;
    }
    src[q] = ptr;
  }
  T rv[5][kRBS / 16];
#pragma unroll
  for (int q = 0; q < 5; ++q)
#pragma unroll
    for (int rr = 0; rr < kRBS / 16; ++rr) {
      const int k = lk + 16 * rr;
      rv[q][rr] = (src[q] && k < nr) ? src[q][r0 + k] : (T)0;
    }
#pragma unroll
  for (int q = 0; q < 5; ++q)
#pragma unroll
    for (int rr = 0; rr < kRBS / 16; ++rr) Ms[cg + 16 * q][lk + 16 * rr] = rv[q][rr];
  __syncthreads();
  acc_t acc[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) acc[c] = acc_t{};
  for (int kk = 0; kk < nr16; kk += 4) {
    const int kr = kk + (lane >> 4);
    const T a = Ms[16 * wv + lr][kr];
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[c] = RbMma<T>::run(a, Ms[16 * c + lr][kr], acc[c]);
  }
  T* P = part + (int64_t)blockIdx.x * (kRBX * kRBY);
#pragma unroll
  for (int c = 0; c < 5; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) P[(16 * wv + RbMma<T>::row(lane, v)) * kRBY + 16 * c + lr] = acc[c][v];
}

// C[i][j] = sum over slices of the partial blocks.  Workgroup = 64 entries;
// wave g adds slices g, g + 4, ... (sixteen loads in flight), then the four
// wave sums are added in wave order (deterministic).
constexpr int kRedDepth = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_rkb_reduce(const T* __restrict__ part, int nslices,
                                                    double* __restrict__ C, const int* inner_done,
                                                    const int* outer_done) {
  if (rb_skip(inner_done, outer_done)) return;
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (e < kRBX * kRBY) {
    for (int s0 = g; s0 < nslices; s0 += 4 * kRedDepth) {
      T v[kRedDepth];
#pragma unroll
      for (int u = 0; u < kRedDepth; ++u) {
        const int sl = s0 + 4 * u;
        v[u] = sl < nslices ? part[(int64_t)sl * (kRBX * kRBY) + e] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < kRedDepth; ++u) acc += (double)v[u];
    }
  }
  red[g][lane] = acc;
  __syncthreads();
  if (g == 0 && e < kRBX * kRBY) C[e] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Broadcast lane `src`'s double to the whole wave (two 32-bit lane reads).
__device__ inline double lane_value(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// The block's scalar recurrences are two lower-triangular solves of size bt:
//   c_{j1(t)} gamma_t + sum_{tau<t} (u_t^T u_tau) gamma_tau = bhat_{j1(t)} - u_t^T w_0
//   c_{j2(t)} delta_t + sum_{tau<t} (v_t^T v_tau) delta_tau
//                     = v_t^T s_0 + sum_{tau<=t} (v_t^T u_tau) gamma_tau.
// One wave: lane tau keeps its row of both systems in registers; step t takes
// lane t's unknown, broadcasts it (lane reads) and every lane subtracts its
// term (column-oriented substitution, no reductions).  z_b then takes, for
// each distinct column b of the block, the sum of its delta_t in step order.
__global__ __launch_bounds__(64) void k_rkb_recur(const double* __restrict__ C, int bt,
                                                   const int* __restrict__ j1, const int* __restrict__ j2,
                                                   const double* __restrict__ tgt, const double* __restrict__ cn,
                                                   double* __restrict__ z, double* __restrict__ coef,
                                                   const int* inner_done, const int* outer_done) {
  if (rb_skip(inner_done, outer_done)) return;
  __shared__ double ds[kRB];
  __shared__ int jb[kRB];
  const double* Cs = C;
  const int lane = threadIdx.x;
  const int tau = lane < kRB ? lane : kRB - 1;  // lanes >= kRB mirror the last row, unused
  const bool live = lane < bt;
  const int a = live ? j1[lane] : 0, b = live ? j2[lane] : 0;
  const double rcg = live ? 1.0 / cn[a] : 0.0;
  const double rcd = live ? 1.0 / cn[b] : 0.0;
  double rg = live ? tgt[a] - Cs[tau * kRBY + kRBX] : 0.0;  // gamma system right-hand side
  double rd = live ? Cs[(kRB + tau) * kRBY + kRBX + 1] : 0.0;  // delta system right-hand side
  double uu[kRB], vu[kRB], vv[kRB];
#pragma unroll
  for (int k = 0; k < kRB; ++k) {
    uu[k] = Cs[tau * kRBY + k];
    vu[k] = Cs[(kRB + tau) * kRBY + k];
    vv[k] = Cs[(kRB + tau) * kRBY + kRB + k];
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
    ds[lane] = del;
    jb[lane] = live ? b : -1;
  }
  __builtin_amdgcn_wave_barrier();
  __threadfence_block();
  if (live) {
    bool first = true;
    for (int u = 0; u < lane; ++u) first = first && jb[u] != b;
    if (first) {
      double sum = 0.0;
      for (int u = lane; u < bt; ++u)
        if (jb[u] == b) sum += ds[u];
      z[b] += sum;
    }
  }
}

// w += sum_t gamma_t u_t, s += sum_t gamma_t u_t - sum_t delta_t v_t.
// Workgroup = 64 rows x 4 quarters of the 2 kRB gathered columns (sixteen
// loads in flight per thread); the quarters are added in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_rkb_update(const T* __restrict__ A1, int64_t lda, int64_t p,
                                                    const int* __restrict__ j1, const int* __restrict__ j2, int bt,
                                                    const double* __restrict__ coef, T* __restrict__ w,
                                                    T* __restrict__ s, const int* inner_done,
                                                    const int* outer_done) {
  if (rb_skip(inner_done, outer_done)) return;
  __shared__ double cf[kRBX];
  __shared__ int64_t off[kRBX];
  __shared__ double part[4][64];
  if (threadIdx.x < kRBX) {
    const int c = threadIdx.x;
    cf[c] = coef[c];
    off[c] = c < kRB ? (c < bt ? (int64_t)j1[c] * lda : 0) : (c - kRB < bt ? (int64_t)j2[c - kRB] * lda : 0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  constexpr int kQ = kRBX / 4;
  double acc = 0.0;
  if (i < p) {
    const T* a = A1 + i;
    T v[kQ];
#pragma unroll
    for (int u = 0; u < kQ; ++u) v[u] = a[off[q * kQ + u]];
#pragma unroll
    for (int u = 0; u < kQ; ++u) acc = fma(cf[q * kQ + u], (double)v[u], acc);
  }
  part[q][lane] = acc;
  __syncthreads();
  if (q == 0 && i < p) {
    const double dw = part[0][lane] + part[1][lane];
    const double dv = part[2][lane] + part[3][lane];
    w[i] = (T)((double)w[i] + dw);
    s[i] = (T)((double)s[i] + (dw - dv));
  }
}

int64_t rk_block_steps() { return kRB; }

size_t rk_block_scratch(int64_t p) {
  // partial blocks of every slice (as doubles) plus C and the coefficients
  const int64_t rows = rk_block_slice_rows(p);
  const int64_t nsl = (p + rows - 1) / rows;
  return (size_t)nsl * kRBX * kRBY + (size_t)kRBX * kRBY + kRBX;
}

int64_t rk_block_slice_rows(int64_t p) {
  int64_t rows = (p + 255) / 256;              // about one slice per CU
  rows = (rows + 15) / 16 * 16;
  if (rows < 16) rows = 16;
  return rows > kRBS ? kRBS : rows;
}

template <typename T>
static void rkb_run(hipStream_t st, const T* A1, int64_t lda, int64_t p, const double* tgt, const double* cn,
                    const int* j1, const int* j2, int64_t count, T* w, T* s, double* z, double* scratch,
                    const int* inner_done, const int* outer_done) {
  const int64_t rows = rk_block_slice_rows(p);
  const int nsl = (int)((p + rows - 1) / rows);
  T* part = (T*)scratch;
  double* C = scratch + (int64_t)nsl * kRBX * kRBY;
  double* coef = C + kRBX * kRBY;
  for (int64_t t0 = 0; t0 < count; t0 += kRB) {
    const int bt = (int)(count - t0 < kRB ? count - t0 : kRB);
    hipLaunchKernelGGL((k_rkb_gram<T>), dim3((unsigned)nsl), dim3(256), 0, st, A1, lda, p, j1 + t0, j2 + t0, bt,
                       (const T*)w, (const T*)s, rows, part, inner_done, outer_done);
    hipLaunchKernelGGL((k_rkb_reduce<T>), dim3((kRBX * kRBY + 63) / 64), dim3(256), 0, st, (const T*)part, nsl,
                       C, inner_done, outer_done);
    hipLaunchKernelGGL(k_rkb_recur, dim3(1), dim3(64), 0, st, (const double*)C, bt, j1 + t0, j2 + t0, tgt, cn, z,
                       coef, inner_done, outer_done);
    hipLaunchKernelGGL((k_rkb_update<T>), dim3((unsigned)((p + 63) / 64)), dim3(256), 0, st, A1, lda, p, j1 + t0,
                       j2 + t0, bt, (const double*)coef, w, s, inner_done, outer_done);
  }
}

void launch_rk_blocks(hipStream_t st, const double* A1, int64_t lda, int64_t p, const double* tgt, const double* cn,
                      const int* j1, const int* j2, int64_t count, double* w, double* s, double* z, double* scratch,
                      const int* inner_done, const int* outer_done) {
  rkb_run<double>(st, A1, lda, p, tgt, cn, j1, j2, count, w, s, z, scratch, inner_done, outer_done);
}

void launch_rk_blocks_f32(hipStream_t st, const float* A1, int64_t lda, int64_t p, const double* tgt,
                          const double* cn, const int* j1, const int* j2, int64_t count, float* w, float* s,
                          double* z, double* scratch, const int* inner_done, const int* outer_done) {
  rkb_run<float>(st, A1, lda, p, tgt, cn, j1, j2, count, w, s, z, scratch, inner_done, outer_done);
}

}  // namespace ils
