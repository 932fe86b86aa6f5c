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

// One or two Gram products in one launch (A1^T A1 and A2^T A2 share the tile
// grid): part 1's workgroups follow part 0's.
struct GramPart {
  const double* A;   // first row of the block
  int64_t K;         // rows
  const double* vb;  // border column (K entries) or null
  int64_t klen;      // rows per K-slice
  int nsplit;        // K-slices (a multiple of kXcds)
  double* G;         // n x n output (column-major, ldg)
  double* gv;        // A^T vb output (n entries) when vb is set
};
struct GramJob {
  GramPart part[2];
  int nparts;
  int n;             // columns of A
  int nc;            // n plus the border column, if any
  int64_t lda, ldg;
  int ntiles;        // lower-triangle tiles of the nc x nc product
  int wg1;           // first workgroup of part 1
  int64_t pbase1;    // part 1's offset in the partial tiles
};

template <typename T, int TM>
__global__ __launch_bounds__(256) void k_gram(GramJob job, T* __restrict__ partials) {
  typedef typename Mma<T>::acc_t acc_t;
  constexpr int NB = TM / 32;       // 16x16 blocks per wave edge
  constexpr int NL = TM / 16;       // loads per thread per operand per stage
  __shared__ T As[2][TM][kGLd];
  __shared__ T Bs[2][TM][kGLd];
  const bool second = job.nparts == 2 && (int)blockIdx.x >= job.wg1;
  const int bid = second ? (int)blockIdx.x - job.wg1 : (int)blockIdx.x;
  const double* A = second ? job.part[1].A : job.part[0].A;
  const int64_t K = second ? job.part[1].K : job.part[0].K;
  const double* vb = second ? job.part[1].vb : job.part[0].vb;
  const int64_t klen = second ? job.part[1].klen : job.part[0].klen;
  if (second) partials += job.pbase1;
  const int64_t lda = job.lda;
  const int n = job.n, ntiles = job.ntiles;
  const int slot = bid / kXcds;
  const int split = (int)(bid % kXcds) + kXcds * (slot / ntiles);
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
__global__ __launch_bounds__(256) void k_gram_finalize(GramJob job, const T* __restrict__ partials) {
  const bool second = (int)blockIdx.y >= job.ntiles;
  const int tile = second ? (int)blockIdx.y - job.ntiles : (int)blockIdx.y;
  const int nsplit = second ? job.part[1].nsplit : job.part[0].nsplit;
  double* G = second ? job.part[1].G : job.part[0].G;
  double* gv = second ? job.part[1].gv : job.part[0].gv;
  if (second) partials += job.pbase1;
  const int ntiles = job.ntiles, n = job.n, nc = job.nc;
  const int64_t ldg = job.ldg;
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

// K-split of one part: about cfg.workgroups workgroups over the tiles, at
// least 256 rows per slice, whole slices per XCD.
static void split_plan(int64_t K, int ntiles, int64_t target, int& nsplit, int64_t& klen) {
  if (K <= 0) {
    nsplit = kXcds;
    klen = kGK;
    return;
  }
  int64_t want = (target + ntiles - 1) / ntiles;
  int64_t maxs = (K + 255) / 256;
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  want = (want + kXcds - 1) / kXcds * kXcds;
  klen = (K + want - 1) / want;
  klen = (klen + kGK - 1) / kGK * kGK;
  nsplit = (int)want;  // trailing slices may be empty: they add zeros
}

static void gram_plan_cfg(int64_t nc, int64_t K, GramCfg cfg, int& tm, int& ntiles, int& nsplit, int64_t& klen) {
  tm = cfg.tile;
  const int nt = (int)((nc + tm - 1) / tm);
  ntiles = nt * (nt + 1) / 2;
  split_plan(K, ntiles, cfg.workgroups, nsplit, klen);
}

// Second part of a two-part launch: slices of about part 0's length.
static void second_plan(int64_t K1, int64_t klen0, int& nsplit, int64_t& klen) {
  if (K1 <= 0) {
    nsplit = kXcds;
    klen = kGK;
    return;
  }
  int64_t want = (K1 + klen0 - 1) / klen0;
  want = (want + kXcds - 1) / kXcds * kXcds;
  klen = (K1 + want - 1) / want;
  klen = (klen + kGK - 1) / kGK * kGK;
  nsplit = (int)want;
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

size_t gram2_partials_size(int64_t n, int64_t K0, int64_t K1) {
  int tm, ntiles, ns0, ns1;
  int64_t kl0, kl1;
  gram_plan_cfg(n + 1, K0, gram_cfg(ILS_PREC_FP64, n, K0), tm, ntiles, ns0, kl0);
  second_plan(K1, kl0, ns1, kl1);
  return std::max((size_t)ntiles * (ns0 + ns1) * tm * tm, gram_partials_size(n, K0));
}

size_t gram_partials_size_cfg(int64_t n, int64_t K, GramCfg c) { return plan_size(n, K, c); }

template <typename T, int TM>
static void gram_launch(hipStream_t s, const GramJob& job, T* partials, hipEvent_t mid) {
  const int wgs = job.ntiles * (job.part[0].nsplit + (job.nparts == 2 ? job.part[1].nsplit : 0));
  hipLaunchKernelGGL((k_gram<T, TM>), dim3(wgs), dim3(256), 0, s, job, partials);
  if (mid) (void)hipEventRecord(mid, s);
  hipLaunchKernelGGL((k_gram_finalize<T, TM>), dim3(TM * TM / 256, job.ntiles * job.nparts), dim3(256), 0, s,
                     job, (const T*)partials);
}

// Gram of rows [0, K) of A with the configuration of (n, K); a border column
// vb (K entries) adds A^T vb, written to gv.  With a second block (K1 rows
// at A1, border vb1) both products come from one launch pair.
template <typename T>
static void gram_run(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda, const double* vb,
                     T* partials, double* G, int64_t ldg, double* gv, hipEvent_t mid, GramCfg cfg,
                     int64_t K1 = -1, const double* A1 = nullptr, const double* vb1 = nullptr,
                     double* G1 = nullptr, double* gv1 = nullptr) {
  GramJob job;
  job.n = (int)n;
  job.nc = (int)n + (vb ? 1 : 0);
  job.lda = lda;
  job.ldg = ldg;
  int tm;
  gram_plan_cfg(job.nc, K, cfg, tm, job.ntiles, job.part[0].nsplit, job.part[0].klen);
  job.part[0] = GramPart{A, K, vb, job.part[0].klen, job.part[0].nsplit, G, gv};
  job.nparts = K1 >= 0 ? 2 : 1;
  job.wg1 = job.ntiles * job.part[0].nsplit;
  job.pbase1 = (int64_t)job.ntiles * job.part[0].nsplit * tm * tm;
  job.part[1] = job.part[0];
  if (job.nparts == 2) {
    int ns1;
    int64_t kl1;
    second_plan(K1, job.part[0].klen, ns1, kl1);
    job.part[1] = GramPart{A1, K1, vb1, kl1, ns1, G1, gv1};
  }
  if (tm == 128)
    gram_launch<T, 128>(s, job, partials, mid);
  else
    gram_launch<T, 64>(s, job, partials, mid);
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

void launch_gram2_f64(hipStream_t s, int64_t n, int64_t lda, int64_t ldg, double* partials, hipEvent_t mid,
                      int64_t K0, const double* A0, const double* vb0, double* G0, double* gv0,
                      int64_t K1, const double* A1, const double* vb1, double* G1, double* gv1) {
  gram_run<double>(s, K0, n, A0, lda, vb0, partials, G0, ldg, gv0, mid, gram_cfg(ILS_PREC_FP64, n, K0), K1, A1,
                   vb1, G1, gv1);
}

void launch_gram_f32(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda,
                     float* partials, double* G, int64_t ldg, hipEvent_t mid) {
  gram_run<float>(s, K, n, A, lda, nullptr, partials, G, ldg, nullptr, mid, gram_cfg(ILS_PREC_MIXED, n, K));
}

}  // namespace ils
