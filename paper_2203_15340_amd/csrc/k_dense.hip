// k_dense.hip -- streaming kernels over the column-major ILS matrix A on
// gfx950: the column pass (A^T J b and squared column norms), the normal
// equation residual, and small vector/matrix helpers.
#include "ils_common.hpp"

namespace ils {

// ------------------------------------------------------------------ column pass
// One workgroup per column j: g_j = A1_(j)^T b1 - A2_(j)^T b2 (Alg. 1 step 4)
// and cn_j = ||A1_(j)||^2, the column weights of Alg. 2 steps 8 and 10.
// Non-finite entries of A or b raise kBitNonfinite.  With a1f, the pass also
// writes A1 rounded to FP32 (leading dimension ldaf), the operand of the
// mixed-precision Gram, while it reads A anyway.
constexpr int kColThreads = 256;

__global__ __launch_bounds__(kColThreads) void k_colpass(const double* __restrict__ A, int64_t lda,
                                                          int64_t p, int64_t q,
                                                          const double* __restrict__ b,
                                                          double* __restrict__ g,
                                                          double* __restrict__ cn, int* bits,
                                                          float* __restrict__ a1f, int64_t ldaf) {
  __shared__ double red[3][kColThreads / kWave];
  const int64_t j = blockIdx.x;
  const double* col = A + j * lda;
  double s1 = 0.0, s2 = 0.0, c = 0.0;
  bool ok = true;
  constexpr int U = 4;  // loads in flight per thread per round
  for (int64_t i0 = 0; i0 < p; i0 += U * kColThreads) {
    double av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + threadIdx.x + u * kColThreads;
      av[u] = i < p ? col[i] : 0.0;
      bv[u] = i < p ? b[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s1 += av[u] * bv[u];
      c += av[u] * av[u];
      ok &= isfinite(av[u]) && isfinite(bv[u]);
    }
    if (a1f) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + threadIdx.x + u * kColThreads;
        if (i < p) a1f[i + j * ldaf] = (float)av[u];
      }
    }
  }
  for (int64_t i0 = p; i0 < p + q; i0 += U * kColThreads) {
    double av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + threadIdx.x + u * kColThreads;
      av[u] = i < p + q ? col[i] : 0.0;
      bv[u] = i < p + q ? b[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s2 += av[u] * bv[u];
      ok &= isfinite(av[u]) && isfinite(bv[u]);
    }
  }
  if (__any(!ok) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(bits, kBitNonfinite);
  s1 = block_sum<kColThreads>(s1, red[0]);
  s2 = block_sum<kColThreads>(s2, red[1]);
  c = block_sum<kColThreads>(c, red[2]);
  if (threadIdx.x == 0) {
    g[j] = s1 - s2;
    if (cn) cn[j] = c;
  }
}

void launch_colpass(hipStream_t s, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                    const double* b, double* g, double* cn, int* bits, float* a1f, int64_t ldaf) {
  hipLaunchKernelGGL(k_colpass, dim3((unsigned)n), dim3(kColThreads), 0, s, A, lda, p, q, b, g, cn,
                     bits, a1f, ldaf);
}

// g = g1 - g2 with g1 = A1^T b1 and g2 = A2^T b2 taken from the bordered Gram
// products, copied into gcol as well.  A non-finite entry of g or of either
// Gram diagonal (a non-finite entry of A or b, or a column whose squares
// overflow) raises kBitNonfinite.
__global__ __launch_bounds__(256) void k_border_combine(int64_t n, double* __restrict__ g,
                                                        const double* __restrict__ g2,
                                                        const double* __restrict__ G1,
                                                        const double* __restrict__ G2, int64_t ldg,
                                                        double* __restrict__ gcol, int* bits) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int bad = 0;
  if (j < n) {
    const double v = g[j] - g2[j];
    g[j] = v;
    gcol[j] = v;
    bad = !isfinite(v) || !isfinite(G1[j + j * ldg]) || !isfinite(G2[j + j * ldg]);
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(bits, kBitNonfinite);
}

void launch_border_combine(hipStream_t s, int64_t n, double* g, const double* g2, const double* G1,
                           const double* G2, int64_t ldg, double* gcol, int* bits) {
  hipLaunchKernelGGL(k_border_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, g, g2, G1, G2,
                     ldg, gcol, bits);
}

// A non-finite diagonal entry of G1 or G2 (a non-finite entry of A, or a
// column whose squares overflow) raises kBitNonfinite.
__global__ __launch_bounds__(256) void k_diag_screen(int64_t n, const double* __restrict__ G1,
                                                     const double* __restrict__ G2, int64_t ldg, int* bits) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int bad = j < n && (!isfinite(G1[j + j * ldg]) || !isfinite(G2[j + j * ldg]));
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(bits, kBitNonfinite);
}

void launch_diag_screen(hipStream_t s, int64_t n, const double* G1, const double* G2, int64_t ldg, int* bits) {
  hipLaunchKernelGGL(k_diag_screen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, G1, G2, ldg, bits);
}

// ------------------------------------------------------------------ residual
// r = A^T J (b - A x); up to n = 1024 in one pass over A (below), otherwise
// in two.
// Pass 1: t = b - A x.  A is column-major, so a wavefront owns 64 rows and
// walks a range of columns (coalesced 512-byte column segments, eight loads
// in flight).  The columns are cut into 4 * ngroups ranges: the four waves of
// a workgroup take four of them and add their partial sums in LDS, and the
// ngroups workgroups per row block write partial vectors that a second kernel
// adds in group order (deterministic).  The column split gives enough
// wavefronts to stream A at HBM rate even when m is small.
constexpr int kResRows = 64;

static int64_t resid_groups(int64_t m, int64_t n) {
  const int64_t rb = (m + kResRows - 1) / kResRows;
  int64_t g = (2048 + rb - 1) / rb;      // aim at ~2048 workgroups
  const int64_t gmax = (n + 31) / 32;    // at least 8 columns per wave
  if (g > gmax) g = gmax;
  return g < 1 ? 1 : g;
}

// One pass over A for n <= kR1MaxN.  A workgroup of 1024 threads takes
// blocks of 16 rows in turn; thread (k = tid % 16, g = tid / 16) holds row k
// of the block at columns g, g + 64, ... (the 16 row lanes of a column read
// one 128-byte segment), forms t_k = b_k - (A x)_k with the other 63 column
// groups through LDS, and adds J_kk t_k A_kc into the column sums, so the
// block is read from memory once.  The next block's loads are issued before
// the current block is reduced (two register sets, one barrier per block
// that waits for LDS only), and the per-block column sums are reduced over
// the 16 row lanes at once, so each thread keeps one accumulator instead of
// 16 (37.3 -> 33.0 us at 20000 x 1000, 4.8 TB/s; mapping blocks to XCDs in
// runs or giving each workgroup a contiguous range of blocks moved it by
// under 1 us).  Each workgroup's column sums go to a partial vector; a
// second kernel adds the partials in workgroup order.
// Partner value for the recursive halving over the 16 row lanes of a DPP
// row at level o (8, 4, 2, 1): a lane whose bit o differs and whose earlier
// levels agree.  The mirror within 16 lanes (level 8) and within 8 lanes
// (level 4) pair such lanes as well as lane ^ o does, and move by DPP
// instead of an LDS permute; levels 2 and 1 are lane ^ 2 and lane ^ 1.
__device__ inline double row_partner(double v, int o) {
  switch (o) {
    case 8: return __builtin_amdgcn_update_dpp(0.0, v, 0x140, 0xF, 0xF, false);  // row_mirror
    case 4: return __builtin_amdgcn_update_dpp(0.0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    case 2: return __builtin_amdgcn_update_dpp(0.0, v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    default: return __builtin_amdgcn_update_dpp(0.0, v, 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
  }
}

constexpr int kR1Threads = 1024;
constexpr int kR1Rows = 16;
constexpr int kR1Groups = kR1Threads / kR1Rows;  // 64 column groups
constexpr int kR1Per = 16;                       // columns per thread
constexpr int64_t kR1MaxN = (int64_t)kR1Groups * kR1Per;
constexpr int kR1Wgs = kResidDefaultWgs;  // one per CU
constexpr int kR1StepsPerRsrc = 4;        // column steps per buffer resource

static int r1_wgs(int64_t m, int wgs) {
  const int64_t nblk = (m + kR1Rows - 1) / kR1Rows;
  return (int)(nblk < wgs ? (nblk > 0 ? nblk : 1) : wgs);
}

static bool one_pass(int64_t n, ResidCfg c) { return n <= kR1MaxN && c.path == kResidAuto; }
// the one-pass kernel's buffer offsets reach (kR1Rows + 4 kR1Groups lda) doubles
static bool one_pass_fits(int64_t lda) {
  return ((int64_t)kR1Rows + (int64_t)kR1StepsPerRsrc * kR1Groups * lda) * 8 < ((int64_t)1 << 31);
}

size_t residual_scratch_cfg(int64_t m, int64_t n, ResidCfg c) {
  const size_t two = (size_t)(resid_groups(m, n) + 1) * (size_t)(m > 0 ? m : 1);
  const size_t one = (size_t)(m > 0 ? m : 1) + (size_t)(c.wgs > 0 ? c.wgs : kR1Wgs) * (size_t)(n > 0 ? n : 1);
  return one_pass(n, c) ? (two > one ? two : one) : two;
}

size_t residual_scratch(int64_t m, int64_t n) {
  const size_t a = residual_scratch_cfg(m, n, ResidCfg{}), b = residual_scratch_cfg(m, n, residual_cfg(n, m));
  return a > b ? a : b;
}

// s_waitcnt lgkmcnt(0) alone (vmcnt and expcnt at their maxima), so a
// barrier can publish LDS writes while global loads stay in flight.
#define ILS_WAIT_LGKM0() __builtin_amdgcn_s_waitcnt((0xF) | (0x3 << 14) | (0x7 << 4))
__device__ inline void lds_barrier() {
  ILS_WAIT_LGKM0();
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ __volatile__("" ::: "memory");
}

struct R1Block {
  double a[kR1Per];
  double b;
};

// The block's loads are buffer loads: one resource (a wave-uniform base) per
// 4 column steps, the step within them as a scalar offset and one 32-bit
// byte offset per lane (k + g lda), so the addresses take no per-load
// registers.  Loads out of range return zero without a branch: columns past
// n lie past the resource's size, and a row past m gets an offset past every
// size.  The launch keeps 4 kR1Groups lda rows within 2^31 bytes.
constexpr int kBufRsrcWord3 = 0x00020000;  // raw (untyped) buffer access on gfx9-family parts
constexpr uint32_t kBufOutOfRange = 0x7fffffffu;

__device__ inline void r1_load(R1Block& d, const double* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                               const double* __restrict__ b, int64_t blk, int k, uint32_t boff) {
  const int64_t i = blk * kR1Rows + k;
  const bool row_ok = i < m;
  d.b = b[row_ok ? i : m - 1];  // first, so its wait is not the last load's; unused past m
  const uint32_t voff = row_ok ? boff : kBufOutOfRange;
#pragma unroll
  for (int u0 = 0; u0 < kR1Per; u0 += kR1StepsPerRsrc) {
    // bytes from this resource's first column to column n
    const int64_t cols = n - (int64_t)kR1Groups * u0;
    const int64_t bytes = cols > 0 ? cols * lda * 8 : 0;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(A + blk * kR1Rows + (int64_t)kR1Groups * u0 * lda), (short)0,
        (int)(bytes < (int64_t)kBufOutOfRange ? bytes : (int64_t)kBufOutOfRange), kBufRsrcWord3);
#pragma unroll
    for (int e = 0; e < kR1StepsPerRsrc; ++e) {
      const int soff = (int)((int64_t)kR1Groups * e * lda * 8);
      d.a[u0 + e] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
    }
  }
}

// First block of workgroup b: the workgroups of one XCD (b % 8, dealt
// round-robin) take consecutive blocks in each round of G (when G is a
// multiple of 8), so an XCD's requests cover adjacent rows of every column.
__device__ inline int64_t r1_first(int64_t b, int64_t G) { return (G % 8) ? b : (b % 8) * (G / 8) + b / 8; }

__global__ __launch_bounds__(kR1Threads) void k_resid_1pass(const double* __restrict__ A, int64_t lda,
                                                             int64_t p, int64_t m, int64_t n,
                                                             const double* __restrict__ b,
                                                             const double* __restrict__ x,
                                                             double* __restrict__ part, const int* done,
                                                             SpStopCheck chk) {
  if (done && *done) return;
  __shared__ double red[2][kR1Threads / kWave][kR1Rows];
  __shared__ double xs[kR1MaxN];
  __shared__ double chk_red[2][kSpThreads / kWave];
  __shared__ int chk_bad[kSpThreads / kWave];
  const int tid = threadIdx.x, k = tid & (kR1Rows - 1), g = tid / kR1Rows;
  const int lane = tid & (kWave - 1), w = tid / kWave;
  const int64_t nblk = (m + kR1Rows - 1) / kR1Rows;
  const int64_t G = gridDim.x;
  const uint32_t boff = (uint32_t)((k + (int64_t)g * lda) * 8);
  for (int c = tid; c < kR1MaxN; c += kR1Threads) xs[c] = c < n ? x[c] : 0.0;
  // the SP steps' stopping tests, by the first kSpThreads threads in the SP
  // step's own order (their loads go out before the block's, so waiting for
  // them does not wait for the block)
  const bool check = chk.part != nullptr, check2 = check && chk.part_next != nullptr;
  double ctot = 0.0, ctot2 = 0.0;
  int cbad = 0;
  if (check && tid < kSpThreads) {
    for (int bkt = tid; bkt < chk.nblk; bkt += kSpThreads) {
      ctot += chk.part[bkt];
      cbad |= chk.pbad[bkt];
      if (check2) ctot2 += chk.part_next[bkt];
    }
  }
  R1Block d0, d1;
  r1_load(d0, A, lda, m, n, b, r1_first(blockIdx.x, G), k, boff);
  if (check && w < kSpThreads / kWave) {
    ctot = wave_sum(ctot);
    ctot2 = wave_sum(ctot2);
    cbad = __any(cbad);
    if (lane == 0) {
      chk_red[0][w] = ctot;
      chk_red[1][w] = ctot2;
      chk_bad[w] = cbad;
    }
  }
  lds_barrier();
  if (check) {
    double tot = chk_red[0][0], tot2 = chk_red[1][0];
    int anybad = chk_bad[0];
#pragma unroll
    for (int q = 1; q < kSpThreads / kWave; ++q) {
      tot += chk_red[0][q];
      tot2 += chk_red[1][q];
      anybad |= chk_bad[q];
    }
    const bool conv = chk.stop_rule != ILS_STOP_FIXED && sp_metric(tot, chk.stop_rule, chk.scal) < chk.tol;
    bool taken = conv || chk.kk == chk.max_outer || anybad;
    if (check2) {
      const bool conv2 = chk.stop_rule != ILS_STOP_FIXED && sp_metric(tot2, chk.stop_rule, chk.scal) < chk.tol;
      taken = taken || conv2 || chk.kk + 1 == chk.max_outer;
    }
    if (blockIdx.x == 0 && tid == 0) *chk.skip = taken ? 1 : 0;
    if (taken) return;
  }
  double acc = 0.0;  // column g + 64 k
  // one block: t_k = J_kk (b_k - (A x)_k) through LDS, then the block's
  // column sums t^T A_blk, each reduced over the 16 row lanes by recursive
  // halving so that lane k keeps column g + 64 k
  auto process = [&](int64_t blk, R1Block& d, int par) {
    double sx = 0.0;
#pragma unroll
    for (int u = 0; u < kR1Per; ++u) sx = fma(d.a[u], xs[g + kR1Groups * u], sx);
    sx += lane_xor16(sx);
    sx += lane_xor32(sx);
    if (lane < kR1Rows) red[par][w][k] = sx;
    lds_barrier();
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < kR1Threads / kWave; ++q) tot += red[par][q][k];
    const int64_t i = blk * kR1Rows + k;
    double tv = 0.0;
    if (i < m) {
      tv = d.b - tot;
      if (i >= p) tv = -tv;  // J = diag(I_p, -I_q)
    }
#pragma unroll
    for (int u = 0; u < kR1Per; ++u) d.a[u] *= tv;
#pragma unroll
    for (int o = kR1Rows / 2, len = kR1Per; o >= 1; o >>= 1, len >>= 1) {
      const bool up = (k & o) != 0;
#pragma unroll
      for (int j = 0; j < len / 2; ++j) {
        const double lo = d.a[j], hi = d.a[j + len / 2];
        const double got = row_partner(up ? lo : hi, o);
        d.a[j] = (up ? hi : lo) + got;
      }
    }
    acc += d.a[0];
  };
  const int64_t first = r1_first(blockIdx.x, G);
  // (blocks past the end load zeros: no branch around a load)
  for (int64_t blk = first; blk < nblk; blk += 2 * G) {
    r1_load(d1, A, lda, m, n, b, blk + G, k, boff);
    process(blk, d0, 0);
    if (blk + G >= nblk) break;
    r1_load(d0, A, lda, m, n, b, blk + 2 * G, k, boff);
    process(blk + G, d1, 1);
  }
  const int64_t c = g + (int64_t)kR1Groups * k;
  if (c < n) part[c * gridDim.x + blockIdx.x] = acc;
}

// r_c = the workgroup partials of column c added by one wave: lane q takes
// partials q, q + 64, ... in order, then a fixed butterfly.
__global__ __launch_bounds__(256) void k_resid_1pass_fin(const double* __restrict__ part, int nwg, int64_t n,
                                                          double* __restrict__ r, const int* done,
                                                          const int* skip) {
  if ((done && *done) || (skip && *skip)) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t c = (int64_t)blockIdx.x * (256 / kWave) + (threadIdx.x >> 6);
  if (c >= n) return;
  double s = 0.0;
  for (int q = lane; q < nwg; q += kWave) s += part[c * nwg + q];
  s = wave_sum(s);
  if (lane == 0) r[c] = s;
}

__global__ __launch_bounds__(256) void k_resid_rows(const double* __restrict__ A, int64_t lda,
                                                     int64_t m, int64_t n, int64_t cw,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ part, const int* done) {
  if (done && *done) return;
  __shared__ double red[4][kResRows];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * kResRows + lane;
  const int64_t j0 = ((int64_t)blockIdx.y * 4 + w) * cw;
  const int64_t j1 = j0 + cw < n ? j0 + cw : n;
  double s = 0.0;
  if (i < m) {
    const double* a = A + i;
    int64_t j = j0;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (; j + 8 <= j1; j += 8) {
      double av[8], xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        av[u] = a[(j + u) * lda];
        xv[u] = x[j + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = fma(av[u], xv[u], acc[u]);
    }
    for (; j < j1; ++j) acc[0] = fma(a[j * lda], x[j], acc[0]);
    s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && i < m) part[(int64_t)blockIdx.y * m + i] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// t = b - sum of the group partials, in group order.
__global__ __launch_bounds__(256) void k_resid_fin(int64_t m, int64_t groups, const double* __restrict__ b,
                                                    const double* __restrict__ part, double* __restrict__ t,
                                                    const int* done) {
  if (done && *done) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
  for (int64_t g = 0; g < groups; ++g) s += part[g * m + i];
  t[i] = b[i] - s;
}

// Sum of x[i] y[i] over i in [i0, i1), thread share of a workgroup of NT
// threads: four loads in flight per thread per round, summed in index order.
template <int NT>
__device__ inline double strided_dot(const double* __restrict__ x, const double* __restrict__ y,
                                     int64_t i0, int64_t i1) {
  double s = 0.0;
  for (int64_t b0 = i0; b0 < i1; b0 += 4 * NT) {
    double xv[4], yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = b0 + threadIdx.x + u * NT;
      xv[u] = i < i1 ? x[i] : 0.0;
      yv[u] = i < i1 ? y[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += xv[u] * yv[u];
  }
  return s;
}

// Pass 2: r_j = A1_(j)^T t1 - A2_(j)^T t2, one workgroup per column.
__global__ __launch_bounds__(kColThreads) void k_resid_cols(const double* __restrict__ A,
                                                             int64_t lda, int64_t p, int64_t q,
                                                             const double* __restrict__ t,
                                                             double* __restrict__ r,
                                                             const int* done) {
  if (done && *done) return;
  __shared__ double red[2][kColThreads / kWave];
  const int64_t j = blockIdx.x;
  const double* col = A + j * lda;
  double s1 = 0.0, s2 = 0.0;
  s1 = strided_dot<kColThreads>(col, t, 0, p);
  s2 = strided_dot<kColThreads>(col, t, p, p + q);
  s1 = block_sum<kColThreads>(s1, red[0]);
  s2 = block_sum<kColThreads>(s2, red[1]);
  if (threadIdx.x == 0) r[j] = s1 - s2;
}

void launch_residual(hipStream_t s, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                     const double* b, const double* x, double* t, double* r, const int* done,
                     const SpStopCheck* chk) {
  launch_residual_cfg(s, p, q, n, A, lda, b, x, t, r, done, residual_cfg(n, p + q), chk);
}

void launch_residual_cfg(hipStream_t s, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                         const double* b, const double* x, double* t, double* r, const int* done, ResidCfg c,
                         const SpStopCheck* chk) {
  const int64_t m = p + q;
  if (m == 0) {  // no rows: r = 0
    launch_fill_vec(s, n, nullptr, r);
    return;
  }
  if (one_pass(n, c) && one_pass_fits(lda)) {
    const int nwg = r1_wgs(m, c.wgs > 0 ? c.wgs : kR1Wgs);
    double* part = t + (m > 0 ? m : 1);
    SpStopCheck none{};
    hipLaunchKernelGGL(k_resid_1pass, dim3((unsigned)nwg), dim3(kR1Threads), 0, s, A, lda, p, m, n, b, x, part,
                       done, chk ? *chk : none);
    hipLaunchKernelGGL(k_resid_1pass_fin, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, (const double*)part, nwg,
                       n, r, done, chk ? (const int*)chk->skip : nullptr);
    return;
  }
  const int64_t groups = resid_groups(m, n);
  const int64_t cw = (n + 4 * groups - 1) / (4 * groups);
  double* part = t + m;
  hipLaunchKernelGGL(k_resid_rows, dim3((unsigned)((m + kResRows - 1) / kResRows), (unsigned)groups), dim3(256),
                     0, s, A, lda, m, n, cw, x, part, done);
  hipLaunchKernelGGL(k_resid_fin, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, m, groups, b,
                     (const double*)part, t, done);
  hipLaunchKernelGGL(k_resid_cols, dim3((unsigned)n), dim3(kColThreads), 0, s, A, lda, p, q, t, r,
                     done);
}

// ------------------------------------------------------------------ helpers
__global__ __launch_bounds__(1024) void k_norm2(int64_t n, const double* __restrict__ v,
                                                double* __restrict__ out) {
  __shared__ double red[1024 / kWave];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s += v[i] * v[i];
  s = block_sum<1024>(s, red);
  if (threadIdx.x == 0) *out = s;
}

void launch_norm2(hipStream_t s, int64_t n, const double* v, double* out) {
  hipLaunchKernelGGL(k_norm2, dim3(1), dim3(1024), 0, s, n, v, out);
}

// The loop state cleared and, with x_ref, ||x_ref||^2 into scal[1] (the
// relative-error denominator): one launch instead of a fill and k_norm2.
__global__ __launch_bounds__(1024) void k_state_reset(LoopState* __restrict__ st, int64_t n,
                                                      const double* __restrict__ x_ref) {
  __shared__ double red[1024 / kWave];
  constexpr int kWords = (int)(sizeof(LoopState) / sizeof(int));
  static_assert(sizeof(LoopState) % sizeof(int) == 0, "LoopState is a whole number of words");
  int* w = (int*)st;
  for (int e = threadIdx.x; e < kWords; e += 1024) w[e] = 0;
  if (!x_ref) return;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s += x_ref[i] * x_ref[i];
  s = block_sum<1024>(s, red);  // its barrier also orders the zeroing before the store below
  if (threadIdx.x == 0) st->scal[1] = s;
}

void launch_state_reset(hipStream_t s, LoopState* st, int64_t n, const double* x_ref) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1024), 0, s, st, n, x_ref);
}

// Y (ncol x n, ldy) = X^T for X n x ncol (ldx), through 32x32 LDS tiles.
__global__ __launch_bounds__(256) void k_transpose(int64_t n, int64_t ncol, const double* __restrict__ X,
                                                   int64_t ldx, double* __restrict__ Y, int64_t ldy) {
  __shared__ double tileb[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + tx, j = j0 + r;
    tileb[r][tx] = (i < n && j < ncol) ? X[i + j * ldx] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + tx, i = i0 + r;
    if (i < n && j < ncol) Y[j + i * ldy] = tileb[tx][r];
  }
}

void launch_transpose(hipStream_t s, int64_t n, int64_t ncol, const double* X, int64_t ldx, double* Y,
                      int64_t ldy) {
  dim3 grid((unsigned)((n + 31) / 32), (unsigned)((ncol + 31) / 32));
  hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, n, ncol, X, ldx, Y, ldy);
}

__global__ void k_copy_cols(int64_t n, int64_t ncol, const double* __restrict__ X, int64_t ldx,
                            double* __restrict__ Y, int64_t ldy) {
  const int64_t j = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Y[i + j * ldy] = X ? X[i + j * ldx] : 0.0;
}

void launch_copy_cols(hipStream_t s, int64_t n, int64_t ncol, const double* X, int64_t ldx, double* Y,
                      int64_t ldy) {
  if (ncol <= 0 || n <= 0) return;
  unsigned gx = (unsigned)((n + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(k_copy_cols, dim3(gx, (unsigned)ncol), dim3(256), 0, s, n, ncol, X, ldx, Y, ldy);
}

void launch_fill_vec(hipStream_t s, int64_t n, const double* src, double* dst) {
  launch_copy_cols(s, n, 1, src, n, dst, n);
}

__global__ void k_eye(int64_t n, double* __restrict__ Y, int64_t ldy) {
  const int64_t j = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Y[i + j * ldy] = (i == j) ? 1.0 : 0.0;
}

void launch_eye(hipStream_t s, int64_t n, double* Y, int64_t ldy) {
  unsigned gx = (unsigned)((n + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(k_eye, dim3(gx, (unsigned)n), dim3(256), 0, s, n, Y, ldy);
}

// H = G1 - G2 (n x n, column-major, all with leading dimension ld)
__global__ void k_sub(int64_t n, const double* __restrict__ X, int64_t ldx, const double* __restrict__ Y,
                      int64_t ldy, double* __restrict__ Z, int64_t ldz) {
  const int64_t j = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Z[i + j * ldz] = X[i + j * ldx] - Y[i + j * ldy];
}

void launch_sub(hipStream_t s, int64_t n, const double* X, int64_t ldx, const double* Y, int64_t ldy,
                double* Z, int64_t ldz) {
  unsigned gx = (unsigned)((n + 255) / 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(k_sub, dim3(gx, (unsigned)n), dim3(256), 0, s, n, X, ldx, Y, ldy, Z, ldz);
}

}  // namespace ils
