// k_gram.hip -- the Gram products A1^T A1 and A2^T A2 (Alg. 1 steps 2-3) on
// the gfx950 matrix cores, FP64 and FP32 (mixed precision), split-K with a
// deterministic reduction.
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "ils_common.hpp"

namespace ils {

// ------------------------------------------------------------------ Gram (MFMA)
// G = A^T A for K rows of A (A1^T A1 or A2^T A2, Alg. 1 steps 2-3).
// Workgroup = one TM x TM tile of the lower triangle of G over one slice of
// the K rows (split-K); its four waves each own a (TM/2)^2 quadrant made of
// MFMA 16x16 blocks.  Columns of A are K-contiguous, so a TM-column x 16-row
// panel of each operand is read with 128-byte coalesced loads into registers
// one stage ahead, then written to the other half of a double-buffered LDS
// area: one barrier per stage.  Slices write partial tiles; a second kernel
// adds them in slice order (deterministic).
constexpr int kGK = 16;        // rows of A per LDS stage
constexpr int kGLd = kGK + 1;  // padded LDS row

template <typename T>
struct Mma;
template <>
struct Mma<double> {
  typedef v4d acc_t;
  __device__ static acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output element v of a lane sits at row (lane/16) + 4v, column lane%16
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mma<float> {
  typedef v4f acc_t;
  __device__ static acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element v of a lane sits at row 4*(lane/16) + v, column lane%16
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

__device__ inline void tile_of(int tile, int& ti, int& tj) {
  int r = (int)((sqrtf(8.0f * (float)tile + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= tile) ++r;
  while (r * (r + 1) / 2 > tile) --r;
  ti = r;
  tj = tile - r * (r + 1) / 2;
}

// Workgroups are dealt to the 8 XCDs round-robin by linear index; the grid
// is laid out so that all tiles of one K-slice land on the same XCD and share
// the A panels of that slice in its L2.  nsplit is a multiple of 8.
constexpr int kXcds = 8;

template <typename T, int TM>
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ A, int64_t lda, int64_t K,
                                              int n, const double* __restrict__ vb, int64_t klen, int ntiles,
                                              T* __restrict__ partials) {
  typedef typename Mma<T>::acc_t acc_t;
  constexpr int NB = TM / 32;       // 16x16 blocks per wave edge
  constexpr int NL = TM / 16;       // loads per thread per operand per stage
  __shared__ T As[2][TM][kGLd];
  __shared__ T Bs[2][TM][kGLd];
  const int slot = blockIdx.x / kXcds;
  const int split = (int)(blockIdx.x % kXcds) + kXcds * (slot / ntiles);
  const int tile = slot % ntiles;
  int ti, tj;
  tile_of(tile, ti, tj);
  const bool diag = ti == tj;
  const int64_t kbeg = (int64_t)split * klen;
  const int64_t kend = kbeg + klen < K ? kbeg + klen : K;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w >> 1) * (TM / 2), wc = (w & 1) * (TM / 2);
  const int lk = t & 15, lc = t >> 4, lr = lane & 15;
  acc_t acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[a][c] = acc_t{};
  const double* Ai = A + (int64_t)ti * TM * lda;
  const double* Aj = A + (int64_t)tj * TM * lda;
  // column c of each operand tile: a column of A, the border column vb
  // (global column n), or zero padding
  const int ci_lim = n - ti * TM, cj_lim = n - tj * TM;
  const double* pa[NL];
  const double* pb[NL];
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int c = lc + 16 * r;
    pa[r] = c < ci_lim ? Ai + (int64_t)c * lda : (c == ci_lim ? vb : nullptr);
    pb[r] = c < cj_lim ? Aj + (int64_t)c * lda : (c == cj_lim ? vb : nullptr);
  }
  T ra[NL], rb[NL];
  auto fetch = [&](int64_t k0) {
    const int64_t k = k0 + lk;
    const bool kin = k < kend;
#pragma unroll
    for (int r = 0; r < NL; ++r) {
      ra[r] = (kin && pa[r]) ? (T)pa[r][k] : (T)0;
      if (!diag) rb[r] = (kin && pb[r]) ? (T)pb[r][k] : (T)0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int r = 0; r < NL; ++r) {
      As[buf][lc + 16 * r][lk] = ra[r];
      if (!diag) Bs[buf][lc + 16 * r][lk] = rb[r];
    }
  };
  if (kbeg < kend) {
    fetch(kbeg);
    stash(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kGK) {
    const bool more = k0 + kGK < kend;
    if (more) fetch(k0 + kGK);
    T(*Ap)[kGLd] = As[buf];
    T(*Bp)[kGLd] = diag ? As[buf] : Bs[buf];
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T fa[NB], fb[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) fa[a] = Ap[wr + a * 16 + lr][kr];
#pragma unroll
      for (int c = 0; c < NB; ++c) fb[c] = Bp[wc + c * 16 + lr][kr];
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[a][c] = Mma<T>::run(fa[a], fb[c], acc[a][c]);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  T* P = partials + ((size_t)split * ntiles + tile) * (TM * TM);
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int c = 0; c < NB; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr + a * 16 + Mma<T>::row(lane, v);
        const int col = wc + c * 16 + lr;
        P[row * TM + col] = acc[a][c][v];
      }
}

// Sum the slices of each tile in slice order and write the tile and its
// mirror image into the full symmetric G (column-major, ldg); with a border
// column, row n of the bordered product (A^T vb) goes to gv.  One element
// per thread; the slice values are loaded together, then added in order.
template <typename T, int TM>
__global__ __launch_bounds__(256) void k_gram_finalize(const T* __restrict__ partials, int nsplit,
                                                       int ntiles, int n, int nc, double* __restrict__ G,
                                                       int64_t ldg, double* __restrict__ gv) {
  const int tile = blockIdx.y;
  int ti, tj;
  tile_of(tile, ti, tj);
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int row = e / TM, col = e % TM;
  const int i = ti * TM + row, j = tj * TM + col;
  if (i >= nc || j >= nc || (ti == tj && row < col) || (i == n && j == n)) return;
  const T* src = partials + (size_t)tile * (TM * TM) + e;
  const size_t stride = (size_t)ntiles * (TM * TM);
  double s = 0.0;
  int sp = 0;
  for (; sp + 8 <= nsplit; sp += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[(size_t)(sp + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += (double)v[u];
  }
  for (; sp < nsplit; ++sp) s += (double)src[(size_t)sp * stride];
  if (i == n) {  // border row: j < n
    gv[j] = s;
    return;
  }
  G[i + (int64_t)j * ldg] = s;
  G[j + (int64_t)i * ldg] = s;
}

// Launch configuration: tile edge and the number of workgroups to aim for
// (the K-split follows from it).  Defaults: 128-tiles when the matrix is
// large enough to give them split-K work for every CU (512 workgroups), else
// 64-tiles (1024 workgroups).  The autotuner (ils_tune_gram) overrides the
// default per (precision, log2 n bucket, log2 K bucket).
static std::mutex g_cfg_mu;
static std::map<uint32_t, GramCfg> g_cfg;

static int log2_bucket(int64_t x) {
  int b = 0;
  while (((int64_t)1 << b) < x) ++b;
  return b;
}

static uint32_t cfg_key(int precision, int64_t n, int64_t K) {
  return ((uint32_t)precision << 16) | ((uint32_t)log2_bucket(n) << 8) | (uint32_t)log2_bucket(K);
}

GramCfg gram_default_cfg(int64_t n) {
  GramCfg c;
  c.tile = n >= 512 ? 128 : 64;
  c.workgroups = c.tile == 128 ? 512 : 1024;
  return c;
}

GramCfg gram_cfg(int precision, int64_t n, int64_t K) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  auto it = g_cfg.find(cfg_key(precision, n, K));
  return it == g_cfg.end() ? gram_default_cfg(n) : it->second;
}

void gram_set_cfg(int precision, int64_t n, int64_t K, GramCfg c) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  g_cfg[cfg_key(precision, n, K)] = c;
}

void gram_clear_cfg() {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  g_cfg.clear();
}

std::vector<GramCfgEntry> gram_cfg_entries() {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  std::vector<GramCfgEntry> out;
  for (const auto& kv : g_cfg) {
    GramCfgEntry e;
    e.precision = (int)(kv.first >> 16);
    e.n_bucket = (int)((kv.first >> 8) & 0xff);
    e.k_bucket = (int)(kv.first & 0xff);
    e.cfg = kv.second;
    out.push_back(e);
  }
  return out;
}

void gram_set_cfg_bucket(int precision, int n_bucket, int k_bucket, GramCfg c) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  g_cfg[((uint32_t)precision << 16) | ((uint32_t)n_bucket << 8) | (uint32_t)k_bucket] = c;
}

static void gram_plan_cfg(int64_t n, int64_t K, GramCfg cfg, int& tm, int& ntiles, int& nsplit, int64_t& klen) {
  tm = cfg.tile;
  const int nt = (int)((n + tm - 1) / tm);
  ntiles = nt * (nt + 1) / 2;
  if (K <= 0) {
    nsplit = kXcds;
    klen = kGK;
    return;
  }
  const int64_t target = cfg.workgroups;
  int64_t want = (target + ntiles - 1) / ntiles;
  int64_t maxs = (K + 255) / 256;               // at least 256 rows per slice
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  want = (want + kXcds - 1) / kXcds * kXcds;  // whole K-slices per XCD
  klen = (K + want - 1) / want;
  klen = (klen + kGK - 1) / kGK * kGK;
  nsplit = (int)want;  // trailing slices may be empty: they add zeros
}

static size_t plan_size(int64_t n, int64_t K, GramCfg c) {
  int tm, ntiles, nsplit;
  int64_t klen;
  gram_plan_cfg(n, K, c, tm, ntiles, nsplit, klen);
  return (size_t)ntiles * nsplit * tm * tm;
}

// Partial-tile scratch in doubles, enough for either precision's
// configuration, with or without a border column.
size_t gram_partials_size(int64_t n, int64_t K) {
  size_t s = 0;
  for (int64_t nc = n; nc <= n + 1; ++nc)
    s = std::max({s, plan_size(nc, K, gram_cfg(ILS_PREC_FP64, n, K)), plan_size(nc, K, gram_cfg(ILS_PREC_MIXED, n, K))});
  return s;
}

size_t gram_partials_size_cfg(int64_t n, int64_t K, GramCfg c) { return plan_size(n, K, c); }

template <typename T, int TM>
static void gram_launch(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda, const double* vb,
                        T* partials, double* G, int64_t ldg, double* gv, hipEvent_t mid, int ntiles, int nsplit,
                        int64_t klen) {
  const int nc = (int)n + (vb ? 1 : 0);
  hipLaunchKernelGGL((k_gram<T, TM>), dim3(ntiles * nsplit), dim3(256), 0, s, A, lda, K, (int)n, vb, klen,
                     ntiles, partials);
  if (mid) (void)hipEventRecord(mid, s);
  hipLaunchKernelGGL((k_gram_finalize<T, TM>), dim3(TM * TM / 256, ntiles), dim3(256), 0, s, partials,
                     nsplit, ntiles, (int)n, nc, G, ldg, gv);
}

// Gram of rows [0, K) of A with the configuration of (n, K); a border column
// vb (K entries) adds A^T vb, written to gv.
template <typename T>
static void gram_run(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda, const double* vb,
                     T* partials, double* G, int64_t ldg, double* gv, hipEvent_t mid, GramCfg cfg) {
  int tm, ntiles, nsplit;
  int64_t klen;
  gram_plan_cfg(n + (vb ? 1 : 0), K, cfg, tm, ntiles, nsplit, klen);
  if (tm == 128)
    gram_launch<T, 128>(s, K, n, A, lda, vb, partials, G, ldg, gv, mid, ntiles, nsplit, klen);
  else
    gram_launch<T, 64>(s, K, n, A, lda, vb, partials, G, ldg, gv, mid, ntiles, nsplit, klen);
}

void launch_gram_cfg(hipStream_t s, int precision, int64_t K, int64_t n, const double* A, int64_t lda,
                     void* partials, double* G, int64_t ldg, GramCfg cfg) {
  if (precision == ILS_PREC_MIXED)
    gram_run<float>(s, K, n, A, lda, nullptr, (float*)partials, G, ldg, nullptr, nullptr, cfg);
  else
    gram_run<double>(s, K, n, A, lda, nullptr, (double*)partials, G, ldg, nullptr, nullptr, cfg);
}

void launch_gram_f64(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda,
                     double* partials, double* G, int64_t ldg, hipEvent_t mid, const double* vb, double* gv) {
  gram_run<double>(s, K, n, A, lda, vb, partials, G, ldg, gv, mid, gram_cfg(ILS_PREC_FP64, n, K));
}

void launch_gram_f32(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda,
                     float* partials, double* G, int64_t ldg, hipEvent_t mid) {
  gram_run<float>(s, K, n, A, lda, nullptr, partials, G, ldg, nullptr, mid, gram_cfg(ILS_PREC_MIXED, n, K));
}

}  // namespace ils
