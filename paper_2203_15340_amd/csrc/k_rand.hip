// k_rand.hip -- kernels of the randomized inner loops on gfx950:
//   * pre-drawing the column indices of SP-RK-RGS (Alg. 2 steps 8 and 10) and
//     the subsets of SP-SCD (Alg. 5 steps 7-8) for a block of inner steps,
//     all steps in parallel (the draws never depend on the iterate);
//   * the inner loops themselves, one workgroup per problem, which are a
//     chain of dependent reductions and cannot be spread across the chip;
//   * the per-outer-step helpers (right-hand side, stop test, update).
#include <type_traits>

#include "ils_common.hpp"
#include "k_rand.hpp"

namespace ils {

__device__ inline int coherent_load(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ samplers
// Inclusive prefix sums in index order by a single thread, so that the
// weighted draw compares against exactly reproducible boundaries.
__global__ void k_prefix(int64_t n, const double* __restrict__ w, int64_t ldw_stride,
                         double* __restrict__ prefix) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    s += w[j * ldw_stride];
    prefix[j] = s;
  }
}

void launch_prefix(hipStream_t s, int64_t n, const double* w, int64_t stride, double* prefix) {
  hipLaunchKernelGGL(k_prefix, dim3(1), dim3(64), 0, s, n, w, stride, prefix);
}

// Smallest j with prefix[j] > u * prefix[n-1]; if rounding leaves none, the
// last index of positive weight.
__device__ inline int weighted_pick(const double* __restrict__ prefix, int64_t n, double u) {
  const double thr = u * prefix[n - 1];
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (prefix[mid] > thr) hi = mid;
    else lo = mid + 1;
  }
  if (lo < n) return (int)lo;
  int64_t j = n - 1;
  while (j > 0 && prefix[j] == prefix[j - 1]) --j;
  return (int)j;
}

// SP-RK-RGS draws for inner steps [t0, t0 + count) of one outer step:
// counter (t, outer, 0, 0), key (seed, tag); j1 from word 0, j2 from word 1.
__global__ __launch_bounds__(256) void k_rk_draw(uint64_t seed, uint64_t outer, int64_t t0,
                                                 int64_t count, const double* __restrict__ prefix,
                                                 int64_t n, int* __restrict__ j1,
                                                 int* __restrict__ j2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint64_t out[4];
  philox4x64_10((uint64_t)(t0 + i), outer, 0, 0, seed, kTagRk, out);
  j1[i] = weighted_pick(prefix, n, u01(out[0]));
  j2[i] = weighted_pick(prefix, n, u01(out[1]));
}

void launch_rk_draw(hipStream_t s, uint64_t seed, uint64_t outer, int64_t t0, int64_t count,
                    const double* prefix, int64_t n, int* j1, int* j2) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_rk_draw, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, seed, outer,
                     t0, count, prefix, n, j1, j2);
}

// SP-SCD draws, one workgroup per inner step.  alpha_t is uniform on {1..n}
// (word 0) unless fixed.  With norm sampling the column is drawn from the
// weights (word 1).  Otherwise tau_t holds the alpha_t indices with the
// smallest keys (SplitMix64 stream seeded with word 2, low index bits
// replaced by the index); the alpha_t-th smallest key is found by an 8-pass
// radix select over LDS histograms (each pass: histogram of the next byte of
// the keys that share the selected prefix, a parallel prefix over the 256
// bins; the passes end once the selected byte holds a single key), and
// tau_t is written as a bitmask, one wave ballot per 64 indices.
__global__ __launch_bounds__(256) void k_scd_draw(uint64_t seed, uint64_t outer, int64_t t0,
                                                  int64_t n, int64_t alpha_opt, int norm_mode,
                                                  const double* __restrict__ prefix,
                                                  int* __restrict__ alpha_out, int* __restrict__ jout,
                                                  uint32_t* __restrict__ mask, int64_t mask_words) {
  __shared__ uint64_t keys[kScdMaxN];
  __shared__ unsigned hist[256];
  __shared__ unsigned wsum[4];
  __shared__ uint64_t sel_prefix;
  __shared__ int64_t sel_rank;
  __shared__ int sel_one;
  __shared__ uint64_t sel_key;
  const int64_t t = blockIdx.x;
  uint64_t out[4];
  philox4x64_10((uint64_t)(t0 + t), outer, 0, 0, seed, kTagScd, out);
  const int64_t alpha = alpha_opt > 0 ? (alpha_opt < n ? alpha_opt : n) : 1 + uniform_below(out[0], n);
  if (threadIdx.x == 0) alpha_out[t] = (int)alpha;
  uint32_t* mrow = mask + t * mask_words;
  if (norm_mode) {
    if (threadIdx.x == 0) jout[t] = weighted_pick(prefix, n, u01(out[1]));
    return;
  }
  if (alpha >= n) {
    for (int64_t wd = threadIdx.x; wd < mask_words; wd += 256) {
      const int64_t lo = wd * 32, cnt = n - lo;
      mrow[wd] = cnt >= 32 ? 0xFFFFFFFFu : ((1u << cnt) - 1u);
    }
    return;
  }
  int b = 1;
  while (b < 63 && ((int64_t)1 << b) < n) ++b;
  for (int64_t s = threadIdx.x; s < n; s += 256) {
    const uint64_t h = mix64(out[2] + (uint64_t)(s + 1) * 0x9E3779B97F4A7C15ull);
    keys[s] = ((h >> b) << b) | (uint64_t)s;
  }
  if (threadIdx.x == 0) {
    sel_prefix = 0;
    sel_rank = alpha - 1;
    sel_one = 0;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    const uint64_t hmask = pass == 0 ? 0ull : (~0ull << (shift + 8));
    hist[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t pre = sel_prefix;
    const int64_t rank = sel_rank;
    for (int64_t s = threadIdx.x; s < n; s += 256) {
      const uint64_t k = keys[s];
      if ((k & hmask) == pre) atomicAdd(&hist[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    // inclusive prefix over the 256 bins (one per thread): within each wave
    // by shifts, then the totals of the lower waves; the one bin whose range
    // [before, before + count) holds the rank continues the selection
    const unsigned h = hist[threadIdx.x];
    unsigned incl = h;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned o = __shfl_up(incl, off, 64);
      if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    for (int q = 0; q < wv; ++q) incl += wsum[q];
    const int64_t before = (int64_t)incl - h;
    if (h > 0 && before <= rank && rank < (int64_t)incl) {
      sel_rank = rank - before;
      sel_prefix = pre | ((uint64_t)threadIdx.x << shift);
      sel_one = h == 1;
    }
    __syncthreads();
    if (sel_one) {
      // the selected byte holds one key: it is the key of rank alpha - 1
      const uint64_t pm = ~0ull << shift, sp = sel_prefix;
      for (int64_t s = threadIdx.x; s < n; s += 256)
        if ((keys[s] & pm) == sp) sel_key = keys[s];
      __syncthreads();
      break;
    }
  }
  const uint64_t thr = sel_one ? sel_key : sel_prefix;  // exact key of rank alpha - 1
  // bit s of tau_t: keys[s] <= thr, 64 bits per wave ballot
  for (int64_t base = 0; base < n; base += 256) {
    const int64_t s = base + threadIdx.x;
    const uint64_t bal = __ballot(s < n && keys[s] <= thr);
    const int64_t w0 = (base + wv * 64) / 32;
    if (lane == 0 && w0 < mask_words) mrow[w0] = (uint32_t)bal;
    if (lane == 1 && w0 + 1 < mask_words) mrow[w0 + 1] = (uint32_t)(bal >> 32);
  }
}

void launch_scd_draw(hipStream_t s, uint64_t seed, uint64_t outer, int64_t t0, int64_t count, int64_t n,
                     int64_t alpha_opt, int norm_mode, const double* prefix, int* alpha, int* jout,
                     uint32_t* mask, int64_t mask_words) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_scd_draw, dim3((unsigned)count), dim3(256), 0, s, seed, outer, t0, n, alpha_opt,
                     norm_mode, prefix, alpha, jout, mask, mask_words);
}

// ------------------------------------------------------------------ RK-RGS inner
// One workgroup runs `count` inner steps of Alg. 2 (steps 8-11) in the
// incremental form: with s = w - A1 z,
//   gamma = (bhat_j1 - A1_(j1)^T w) / c_j1,  w += gamma A1_(j1),  s += gamma A1_(j1)
//   delta = A1_(j2)^T s / c_j2,  z_j2 += delta,  s -= delta A1_(j2).
// Each thread owns the rows i = tid + e * 1024 of w and s, so the only
// synchronisation is the two block reductions per step.
constexpr int kRkThreads = 1024;

// T = double (FP64 path) or float (mixed precision: FP32 copy of A1, FP32 w
// and s, FP32 sums; z and the right-hand side stay FP64).
template <typename T>
__global__ __launch_bounds__(kRkThreads) void k_rk_inner(const T* __restrict__ A1, int64_t lda,
                                                         int64_t p, const double* __restrict__ tgt,
                                                         const double* __restrict__ cn,
                                                         const int* __restrict__ j1s,
                                                         const int* __restrict__ j2s, int64_t count,
                                                         T* __restrict__ w, T* __restrict__ s,
                                                         double* __restrict__ z,
                                                         const int* inner_done, const int* outer_done) {
  if (*(volatile const int*)inner_done || *(volatile const int*)outer_done) return;
  __shared__ T red[2][kRkThreads / kWave];
  const int tid = threadIdx.x;
  for (int64_t t = 0; t < count; ++t) {
    const int j1 = j1s[t], j2 = j2s[t];
    const T* a1 = A1 + (int64_t)j1 * lda;
    const T* a2 = A1 + (int64_t)j2 * lda;
    T d = 0;
    for (int64_t i = tid; i < p; i += kRkThreads) d += a1[i] * w[i];
    d = block_sum<kRkThreads>(d, red[0]);
    const T gam = (T)((tgt[j1] - (double)d) / cn[j1]);
    T d2 = 0;
    for (int64_t i = tid; i < p; i += kRkThreads) {
      const T av = a1[i];
      w[i] += gam * av;
      const T sv = s[i] + gam * av;
      s[i] = sv;
      d2 += a2[i] * sv;
    }
    d2 = block_sum<kRkThreads>(d2, red[1]);
    const T del = (T)((double)d2 / cn[j2]);
    if (tid == 0) z[j2] += (double)del;
    for (int64_t i = tid; i < p; i += kRkThreads) s[i] -= del * a2[i];
  }
}

void launch_rk_inner(hipStream_t st, const double* A1, int64_t lda, int64_t p, const double* tgt,
                     const double* cn, const int* j1, const int* j2, int64_t count, double* w, double* s,
                     double* z, const int* inner_done, const int* outer_done) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_rk_inner<double>, dim3(1), dim3(kRkThreads), 0, st, A1, lda, p, tgt, cn, j1, j2, count,
                     w, s, z, inner_done, outer_done);
}

void launch_rk_inner_f32(hipStream_t st, const float* A1, int64_t lda, int64_t p, const double* tgt,
                         const double* cn, const int* j1, const int* j2, int64_t count, float* w, float* s,
                         double* z, const int* inner_done, const int* outer_done) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_rk_inner<float>, dim3(1), dim3(kRkThreads), 0, st, A1, lda, p, tgt, cn, j1, j2, count,
                     w, s, z, inner_done, outer_done);
}

// FP32 copy of A1 (p x n, leading dimension p) for the mixed inner sweeps.
__global__ void k_to_f32(int64_t p, int64_t n, const double* __restrict__ A, int64_t lda, float* __restrict__ Af) {
  const int64_t total = p * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t j = e / p, i = e - j * p;
    Af[e] = (float)A[i + j * lda];
  }
}

void launch_to_f32(hipStream_t s, int64_t p, int64_t n, const double* A, int64_t lda, float* Af) {
  int64_t b = (p * n + 255) / 256;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)b), dim3(256), 0, s, p, n, A, lda, Af);
}

// Inner stop test of SP-RK-RGS: ||bhat - A1^T (w - s)|| <= tol * ||bhat||
// (A1 z = w - s).  Pass 1 forms v = w - s, pass 2 is one workgroup per
// column; the last workgroup adds the squared entries in column order.
template <typename T>
__global__ void k_sub_vec(int64_t p, const T* __restrict__ w, const T* __restrict__ s,
                          double* __restrict__ v, const int* skip) {
  if (*(volatile const int*)skip) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = (double)w[i] - (double)s[i];
}

__global__ __launch_bounds__(256) void k_rk_check(const double* __restrict__ A1, int64_t lda, int64_t p,
                                                  int64_t n, const double* __restrict__ v,
                                                  const double* __restrict__ tgt,
                                                  double* __restrict__ res2, double itol2,
                                                  const double* tn2, int* inner_done, unsigned* arrive,
                                                  const int* skip) {
  if (*(volatile const int*)skip) return;
  __shared__ double red[4];
  __shared__ int is_last;
  const int64_t j = blockIdx.x;
  const double* col = A1 + j * lda;
  double sacc = 0.0;
  // eight loads of each operand in flight per thread per round; the sum
  // runs over the rows in the same order as one row at a time
  constexpr int U = 8;
  for (int64_t i0 = 0; i0 < p; i0 += U * 256) {
    double av[U], vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + threadIdx.x + u * 256;
      av[u] = i < p ? col[i] : 0.0;
      vv[u] = i < p ? v[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) sacc += av[u] * vv[u];
  }
  sacc = block_sum<256>(sacc, red);
  if (threadIdx.x == 0) {
    const double rj = tgt[j] - sacc;
    // device-scope store, then wait for it before counting the arrival: the
    // last workgroup reads every entry with device-scope loads (no fence)
    __hip_atomic_store(res2 + j, rj * rj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    is_last = __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last) return;
  double tot = 0.0;
  for (int64_t jj = threadIdx.x; jj < n; jj += 256)
    tot += __hip_atomic_load(res2 + jj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  tot = block_sum<256>(tot, red);
  if (threadIdx.x == 0) {
    *arrive = 0;
    if (tot <= itol2 * (*tn2)) *inner_done = 1;
  }
}

void launch_rk_check(hipStream_t st, const double* A1, int64_t lda, int64_t p, int64_t n, const double* w,
                     const double* s, double* v, const double* tgt, double* res2, double itol2,
                     const double* tn2, int* inner_done, unsigned* arrive, const int* skip) {
  hipLaunchKernelGGL(k_sub_vec<double>, dim3(64), dim3(256), 0, st, p, w, s, v, skip);
  hipLaunchKernelGGL(k_rk_check, dim3((unsigned)n), dim3(256), 0, st, A1, lda, p, n, (const double*)v, tgt,
                     res2, itol2, tn2, inner_done, arrive, skip);
}

void launch_rk_check_f32(hipStream_t st, const double* A1, int64_t lda, int64_t p, int64_t n, const float* w,
                         const float* s, double* v, const double* tgt, double* res2, double itol2,
                         const double* tn2, int* inner_done, unsigned* arrive, const int* skip) {
  hipLaunchKernelGGL(k_sub_vec<float>, dim3(64), dim3(256), 0, st, p, w, s, v, skip);
  hipLaunchKernelGGL(k_rk_check, dim3((unsigned)n), dim3(256), 0, st, A1, lda, p, n, (const double*)v, tgt,
                     res2, itol2, tn2, inner_done, arrive, skip);
}

// ------------------------------------------------------------------ SCD inner
// Inner steps of Alg. 5 (steps 7-11): before each step ||r||^2 (stop test)
// and, over the members of tau_t, the entry of largest |r| (smallest index on
// ties); then r -= r_j / G1_jj * G1_(j) and beta_j += r_j / G1_jj.  With
// norm-weighted sampling (SP-RCD) the pre-drawn index is the only member.
// T is the precision of G1 and r (double; float under mixed precision, where
// the sums are FP32 too); beta is always FP64.

// The better of two candidates (|r|, index): larger |r|, then smaller index.
__device__ inline bool better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}
// The same test with both comparisons evaluated (no branch).
__device__ inline bool better_nb(double v, int i, double bv, int bi) {
  return (v > bv) | ((v == bv) & (i < bi));
}

// Global-memory form for n > kScdMaxN (greedy or norm-weighted choice only):
// one workgroup, r in global memory.
constexpr int kScdThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kScdThreads) void k_scd_inner(
    const T* __restrict__ G1, int64_t ldg, int64_t n, T* __restrict__ r,
    double* __restrict__ beta, const uint32_t* __restrict__ mask, int64_t mask_words,
    const int* __restrict__ jpre, int norm_mode, int64_t count, int check, double itol2,
    const double* tn2, int* inner_done, int64_t* steps_done, const int* outer_done) {
  if (*(volatile const int*)inner_done || *(volatile const int*)outer_done) return;
  __shared__ T red_n[2][kScdThreads / kWave];
  __shared__ double red_v[2][kScdThreads / kWave];
  __shared__ T red_r[2][kScdThreads / kWave];
  __shared__ int red_i[2][kScdThreads / kWave];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double stop2 = itol2 * (*tn2);
  int64_t t = 0;
  for (; t <= count; ++t) {
    const int par = (int)(t & 1);
    const uint32_t* mrow = mask + t * mask_words;
    const int jn = (norm_mode && t < count) ? jpre[t] : -1;
    T nrm = 0;
    double bv = -1.0;
    T br = 0;
    int bi = 0x7FFFFFFF;
    for (int64_t sidx = tid; sidx < n; sidx += kScdThreads) {
      const T rv = r[sidx];
      nrm += rv * rv;
      const bool member = t < count && (norm_mode ? sidx == jn : ((mrow[sidx >> 5] >> (sidx & 31)) & 1u));
      if (member) {
        const double av = norm_mode ? 0.0 : fabs((double)rv);
        if (better(av, (int)sidx, bv, bi)) {
          bv = av;
          br = rv;
          bi = (int)sidx;
        }
      }
    }
    // wave reduction (fixed butterfly), then across waves in wave order
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      nrm += __shfl_xor(nrm, off, kWave);
      const double ov = __shfl_xor(bv, off, kWave);
      const T orr = __shfl_xor(br, off, kWave);
      const int oi = __shfl_xor(bi, off, kWave);
      if (better(ov, oi, bv, bi)) {
        bv = ov;
        br = orr;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_n[par][wv] = nrm;
      red_v[par][wv] = bv;
      red_r[par][wv] = br;
      red_i[par][wv] = bi;
    }
    __syncthreads();
    nrm = red_n[par][0];
    bv = red_v[par][0];
    br = red_r[par][0];
    bi = red_i[par][0];
    for (int q = 1; q < kScdThreads / kWave; ++q) {
      nrm += red_n[par][q];
      if (better(red_v[par][q], red_i[par][q], bv, bi)) {
        bv = red_v[par][q];
        br = red_r[par][q];
        bi = red_i[par][q];
      }
    }
    if (check && (double)nrm <= stop2) {
      if (tid == 0) *inner_done = 1;
      break;
    }
    if (t == count) break;
    const int j = bi;
    if (j < 0 || j >= n) break;  // no finite candidate: the outer update flags it
    __syncthreads();  // everyone has read r before it is overwritten
    const T gam = br / G1[(int64_t)j * ldg + j];
    const T* col = G1 + (int64_t)j * ldg;
    for (int64_t sidx = tid; sidx < n; sidx += kScdThreads) r[sidx] -= gam * col[sidx];
    if (tid == 0) beta[j] += (double)gam;
  }
  if (tid == 0) *steps_done += (t < count ? t : count);
}

// Register form for n <= kScdMaxN.  256 threads; thread th owns E entries
// of r in registers (E = 4, 8 or 16 for n up to 1024, 2048, 4096): the
// consecutive [th E, th E + E) for E = 4, and th, th + 256, ...,
// th + 256 (E - 1) above (a wave's loads of a column then stay contiguous;
// n = 4000: 4.6 -> 3.8 us per step, while at E = 4 the one mask word per
// thread of the consecutive form measured faster), and the matching E bits of
// the step's subset mask, fetched one step ahead (the subsets do not depend
// on r).  A step is:
// the thread's own sum of squares and best member, a butterfly over the
// wave, one barrier, the four wave partials combined in wave order; then
// G1_jj from LDS and the thread's E entries of the column G1_(j) from global
// memory, and the update.  beta lives in LDS for the launch.  Sums, argmax
// and update follow the same definitions as the global-memory form.
constexpr int kScdRegThreads = 256;
constexpr int kScdRegWaves = kScdRegThreads / kWave;

template <typename T, int E>
__global__ __launch_bounds__(kScdRegThreads) void k_scd_inner_reg(
    const T* __restrict__ G1, int64_t ldg, int64_t n, T* __restrict__ r,
    double* __restrict__ beta, const uint32_t* __restrict__ mask, int64_t mask_words,
    const int* __restrict__ jpre, int norm_mode, int64_t count, int check, double itol2,
    const double* tn2, int* inner_done, int64_t* steps_done, const int* outer_done) {
  if (*(volatile const int*)inner_done || *(volatile const int*)outer_done) return;
  __shared__ T dg[kScdMaxN];
  __shared__ double bs[kScdMaxN];
  __shared__ T red_n[2][kScdRegWaves];
  __shared__ double red_v[2][kScdRegWaves];
  __shared__ T red_r[2][kScdRegWaves];
  __shared__ int red_i[2][kScdRegWaves];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const auto gG = glb(G1);
  constexpr bool strided = E > 4;
  auto ix = [&](int e) -> int64_t {
    return strided ? (int64_t)tid + (int64_t)e * kScdRegThreads : (int64_t)tid * E + e;
  };
  T rr[E];
#pragma unroll
  for (int e = 0; e < E; ++e) rr[e] = (ix(e) < n) ? r[ix(e)] : (T)0;
  for (int64_t i = tid; i < n; i += kScdRegThreads) {
    dg[i] = gG[i * ldg + i];
    bs[i] = beta[i];
  }
  __syncthreads();
  const double stop2 = itol2 * (*tn2);
  // this thread's E subset bits for step tt (bit e: entry ix(e))
  auto fetch_bits = [&](int64_t tt) -> uint32_t {
    if (norm_mode || tt >= count) return 0u;
    if constexpr (!strided) {
      // E divides 32: the E bits lie in one word
      const int64_t s0 = ix(0);
      if (s0 >= n) return 0u;
      const uint32_t w0 = mask[tt * mask_words + (s0 >> 5)];
      return (w0 >> (s0 & 31)) & ((1u << E) - 1u);
    }
    uint32_t wd[E];
#pragma unroll
    for (int e = 0; e < E; ++e) wd[e] = ix(e) < n ? mask[tt * mask_words + (ix(e) >> 5)] : 0u;
    uint32_t b = 0u;
#pragma unroll
    for (int e = 0; e < E; ++e) b |= ((wd[e] >> (ix(e) & 31)) & 1u) << e;
    return b;
  };
  uint32_t bits_next = fetch_bits(0);
  int jn_next = (norm_mode && count > 0) ? jpre[0] : -1;
  int64_t t = 0;
  for (; t <= count; ++t) {
    const int par = (int)(t & 1);
    const uint32_t bits = bits_next;
    const int jn = jn_next;
    bits_next = fetch_bits(t + 1);
    jn_next = (norm_mode && t + 1 < count) ? jpre[t + 1] : -1;
    T nrm = 0;
    double bv = -1.0;
    T br = 0;
    int bi = 0x7FFFFFFF;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      nrm += rr[e] * rr[e];
      const bool member = t < count && ix(e) < n && (norm_mode ? ix(e) == jn : ((bits >> e) & 1u));
      const double av = norm_mode ? 0.0 : fabs((double)rr[e]);
      const bool take = member & better_nb(av, (int)ix(e), bv, bi);
      bv = take ? av : bv;
      br = take ? rr[e] : br;
      bi = take ? (int)ix(e) : bi;
    }
    // the wave's sum and best (|r|, index) by DPP moves, selects instead of
    // branches: within each row of 16 lanes the partner lanes are lane ^ 1,
    // lane ^ 2, then the mirror within 8 and within 16 lanes (every lane
    // ends with its row's result); then lane 15 of rows 0 and 2 goes to rows
    // 1 and 3, and lane 31 to rows 2 and 3, so lane 63 holds the wave's
    // result.  Lanes a move does not write get the identity (0, -1, max).
    auto level = [&](auto ctrl, auto rows) {
      constexpr int C = decltype(ctrl)::value, RM = decltype(rows)::value;
      const T on = __builtin_amdgcn_update_dpp((T)0, nrm, C, RM, 0xF, false);
      const double ov = __builtin_amdgcn_update_dpp(-1.0, bv, C, RM, 0xF, false);
      const T orr = __builtin_amdgcn_update_dpp((T)0, br, C, RM, 0xF, false);
      const int oi = __builtin_amdgcn_update_dpp(0x7FFFFFFF, bi, C, RM, 0xF, false);
      nrm += on;
      const bool take = better_nb(ov, oi, bv, bi);
      bv = take ? ov : bv;
      br = take ? orr : br;
      bi = take ? oi : bi;
    };
    level(std::integral_constant<int, 0xB1>{}, std::integral_constant<int, 0xF>{});   // quad_perm 1,0,3,2
    level(std::integral_constant<int, 0x4E>{}, std::integral_constant<int, 0xF>{});   // quad_perm 2,3,0,1
    level(std::integral_constant<int, 0x141>{}, std::integral_constant<int, 0xF>{});  // row_half_mirror
    level(std::integral_constant<int, 0x140>{}, std::integral_constant<int, 0xF>{});  // row_mirror
    level(std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xA>{});  // row_bcast:15
    level(std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xC>{});  // row_bcast:31
    if (lane == 63) {
      red_n[par][wv] = nrm;
      red_v[par][wv] = bv;
      red_r[par][wv] = br;
      red_i[par][wv] = bi;
    }
    __syncthreads();
    nrm = red_n[par][0];
    bv = red_v[par][0];
    br = red_r[par][0];
    bi = red_i[par][0];
#pragma unroll
    for (int q = 1; q < kScdRegWaves; ++q) {
      nrm += red_n[par][q];
      const bool take = better_nb(red_v[par][q], red_i[par][q], bv, bi);
      bv = take ? red_v[par][q] : bv;
      br = take ? red_r[par][q] : br;
      bi = take ? red_i[par][q] : bi;
    }
    if (check && (double)nrm <= stop2) {
      if (tid == 0) *inner_done = 1;
      break;
    }
    if (t == count) break;
    const int j = bi;
    if (j < 0 || j >= n) break;  // no finite candidate: the outer update flags it
    const auto col = gG + (int64_t)j * ldg;
    T cv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) cv[e] = (ix(e) < n) ? col[ix(e)] : (T)0;
    const T gam = br / dg[j];
#pragma unroll
    for (int e = 0; e < E; ++e) rr[e] -= gam * cv[e];
    if (tid == 0) bs[j] += (double)gam;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (ix(e) < n) r[ix(e)] = rr[e];
  for (int64_t i = tid; i < n; i += kScdRegThreads) beta[i] = bs[i];
  if (tid == 0) *steps_done += (t < count ? t : count);
}

template <typename T>
static void scd_inner_run(hipStream_t st, const T* G1, int64_t ldg, int64_t n, T* r, double* beta,
                          const uint32_t* mask, int64_t mask_words, const int* jpre, int norm_mode,
                          int64_t count, int check, double itol2, const double* tn2, int* inner_done,
                          int64_t* steps_done, const int* outer_done) {
#define ILS_SCD_REG(E)                                                                                     \
  hipLaunchKernelGGL((k_scd_inner_reg<T, E>), dim3(1), dim3(kScdRegThreads), 0, st, G1, ldg, n, r, beta, \
                     mask, mask_words, jpre, norm_mode, count, check, itol2, tn2, inner_done, steps_done,  \
                     outer_done)
  if (n <= 4 * kScdRegThreads)
    ILS_SCD_REG(4);
  else if (n <= 8 * kScdRegThreads)
    ILS_SCD_REG(8);
  else if (n <= kScdMaxN)
    ILS_SCD_REG(16);
  else
    hipLaunchKernelGGL((k_scd_inner<T>), dim3(1), dim3(kScdThreads), 0, st, G1, ldg, n, r, beta, mask,
                       mask_words, jpre, norm_mode, count, check, itol2, tn2, inner_done, steps_done,
                       outer_done);
#undef ILS_SCD_REG
}
static_assert(16 * kScdRegThreads == kScdMaxN, "register form covers n <= kScdMaxN");

void launch_scd_inner(hipStream_t st, const double* G1, int64_t ldg, int64_t n, double* r, double* beta,
                      const uint32_t* mask, int64_t mask_words, const int* jpre, int norm_mode,
                      int64_t count, int check, double itol2, const double* tn2, int* inner_done,
                      int64_t* steps_done, const int* outer_done) {
  scd_inner_run<double>(st, G1, ldg, n, r, beta, mask, mask_words, jpre, norm_mode, count, check, itol2, tn2,
                        inner_done, steps_done, outer_done);
}

void launch_scd_inner_f32(hipStream_t st, const float* G1, int64_t ldg, int64_t n, float* r, double* beta,
                          const uint32_t* mask, int64_t mask_words, const int* jpre, int norm_mode,
                          int64_t count, int check, double itol2, const double* tn2, int* inner_done,
                          int64_t* steps_done, const int* outer_done) {
  scd_inner_run<float>(st, G1, ldg, n, r, beta, mask, mask_words, jpre, norm_mode, count, check, itol2, tn2,
                       inner_done, steps_done, outer_done);
}

// ------------------------------------------------------------------ outer helpers
// y = G x + g for symmetric G (column i = row i), one wave per row.
__global__ __launch_bounds__(256) void k_symv_add(int64_t n, const double* __restrict__ G, int64_t ldg,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ g, double* __restrict__ y,
                                                  const int* skip) {
  if (*(volatile const int*)skip) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const double* gc = G + i * ldg;
  double sacc = 0.0;
  for (int64_t j = lane; j < n; j += kWave) sacc += gc[j] * x[j];
  sacc = wave_sum(sacc);
  if (lane == 0) y[i] = sacc + g[i];
}

void launch_symv_add(hipStream_t s, int64_t n, const double* G, int64_t ldg, const double* x,
                     const double* g, double* y, const int* skip) {
  hipLaunchKernelGGL(k_symv_add, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, G, ldg, x, g, y, skip);
}

// Stop test at x_k for the randomized methods (same rules as the SP step):
// metric from x_ref or from the residual r_k; ||target||^2 for the inner test.
__global__ __launch_bounds__(1024) void k_outer_test(int64_t n, const double* __restrict__ xk,
                                                     const double* __restrict__ x_ref,
                                                     const double* __restrict__ rk, int stop_rule,
                                                     double tol, int64_t k, int64_t max_outer,
                                                     LoopState* st) {
  if (st->done || st->bits) return;
  __shared__ double red[1024 / kWave];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    if (stop_rule == ILS_STOP_XREF) {
      const double d = xk[i] - x_ref[i];
      a += d * d;
    } else if (stop_rule == ILS_STOP_RR) {
      a += rk[i] * rk[i];
    }
  }
  a = block_sum<1024>(a, red);
  if (threadIdx.x != 0) return;
  double metric = 0.0;
  if (stop_rule == ILS_STOP_XREF) metric = sqrt(a) / sqrt(st->scal[1]);
  else if (stop_rule == ILS_STOP_RR) metric = a / st->scal[0];
  if (stop_rule != ILS_STOP_FIXED && metric < tol) {
    st->metric = metric;
    st->status = ILS_OK;
    st->iters = k;
    st->done = 1;
  } else if (k == max_outer) {
    st->metric = metric;
    st->status = stop_rule == ILS_STOP_FIXED ? ILS_OK : ILS_ERR_NO_CONVERGENCE;
    st->iters = k;
    st->done = 1;
  }
}

void launch_outer_test(hipStream_t s, int64_t n, const double* xk, const double* x_ref, const double* rk,
                       int stop_rule, double tol, int64_t k, int64_t max_outer, LoopState* st) {
  hipLaunchKernelGGL(k_outer_test, dim3(1), dim3(1024), 0, s, n, xk, x_ref, rk, stop_rule, tol, k,
                     max_outer, st);
}

// x_{k+1} = z (paper form) or x_k + z (correction form); a non-finite entry
// ends the loop with ILS_ERR_NONFINITE at k + 1.
__global__ __launch_bounds__(1024) void k_outer_update(int64_t n, const double* __restrict__ xk,
                                                       const double* __restrict__ z, int correction,
                                                       double* __restrict__ xn, int64_t k, LoopState* st) {
  if (st->done || st->bits) return;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int mybad = 0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double v = correction ? xk[i] + z[i] : z[i];
    xn[i] = v;
    mybad |= !isfinite(v);
  }
  if (mybad) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0 && bad) {
    st->status = ILS_ERR_NONFINITE;
    st->iters = k + 1;
    st->done = 1;
  }
}

void launch_outer_update(hipStream_t s, int64_t n, const double* xk, const double* z, int correction,
                         double* xn, int64_t k, LoopState* st) {
  hipLaunchKernelGGL(k_outer_update, dim3(1), dim3(1024), 0, s, n, xk, z, correction, xn, k, st);
}

__global__ void k_diag(int64_t n, const double* __restrict__ G, int64_t ldg, double* __restrict__ d) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = G[i * ldg + i];
}

void launch_diag(hipStream_t s, int64_t n, const double* G, int64_t ldg, double* d) {
  hipLaunchKernelGGL(k_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, G, ldg, d);
}

__global__ void k_zero_cnt(int64_t n, const double* __restrict__ c, int* bits) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!(c[i] > 0.0)) atomicOr(bits, kBitNotSpd);
}

void launch_zero_col_check(hipStream_t s, int64_t n, const double* c, int* bits) {
  hipLaunchKernelGGL(k_zero_cnt, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, c, bits);
}

}  // namespace ils
