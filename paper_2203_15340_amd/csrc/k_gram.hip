// k_gram.hip -- the Gram products A1^T A1 and A2^T A2 (Alg. 1 steps 2-3) on
// the gfx950 matrix cores, FP64 and FP32 (mixed precision), split-K with a
// deterministic reduction.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
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

// ------------------------------------------------------------------ persistent Gram
// The same lower 64 x 64 tiles, but a fixed grid of kPersWpc workgroups per CU
// that stays resident.  The rows of A are cut into one range per XCD (the
// grid's workgroups are dealt to the XCDs round-robin, so workgroup b runs on
// XCD b % 8 and all tiles of a range share that XCD's L2).  Inside a range,
// workgroup j of the XCD first takes the whole range for tiles j, j + W, ...
// (the q = T / W main tiles per workgroup; all workgroups walk the rows in
// step, so each stage of the panels is fetched into the L2 once and shared),
// then an equal contiguous share of the (tile, stage) pairs of the
// L = T - q W leftover tiles, tile-major.  Every workgroup does the same
// number of stages, with no tail of partly filled rounds.
//
// Operand panels go from global memory straight into LDS
// (global_load_lds_dwordx4: each lane moves 16 bytes, a wave 1 KB, with no
// register staging and no LDS store instructions), two stages in flight.  A
// stage holds, per operand, 64 column slots of RS rows = 8 chunks of 16 bytes
// (RS = 16 rows of FP64, 32 of FP32); chunk q of slot s sits at position
// q ^ ((s >> 1) & 7), so the 16 lanes of an FP64 MFMA operand read (16
// slots, one row) hit 16 distinct bank groups.  A stage that does not start
// on a 16-byte boundary or is shorter than RS rows (a range end, the A1/A2
// boundary) goes through registers into the same layout.  Needs A and the
// border column 16-byte aligned and lda a multiple of 16 bytes.
//
// The FP32 instance reads an FP32 copy of the rows (made by k_copy_f32), so a
// stage carries twice the rows for the same bytes.  Its 4-byte operand reads
// see 2-way bank conflicts (half the LDS cycles); reading 16-byte chunks and
// feeding 4 MFMAs from each removes them but was not faster (211.7 against
// 209.0 us at 18000 x 1000), nor were 5 workgroups per CU (212.9 us): the
// kernel runs at 0.55 of the FP32 MFMA peak, MFMA busy 0.65.
//
// Each share (tile, XCD range, part) writes one partial tile; the reduction
// kernel adds, per tile and part, the shares of XCD 0..7 in row order.
constexpr int kPersWpc = kGramPersistentWpc;  // resident workgroups per CU (32 KB of LDS each)
constexpr int kPersAlign = 16;  // row ranges start on multiples of 16 rows
constexpr int kPersMaxShares = 64;  // shares per (leftover tile, XCD) the reduction lists

enum { kGramTri = 0, kGramRect = 1, kGramWhole = 2 };  // products of the persistent kernel

struct GramPJob {
  const void* A;     // row 0 of the rows [0, M) (double, or float for the FP32 kind)
  int64_t lda;
  const void* vb;    // border column (M entries) or null
  int64_t M, p;      // rows; part 0 = rows [0, p), part 1 = rows [p, M)
  int n, nc, T;      // columns, bordered columns, lower tiles
  int W;             // workgroups per XCD
  int q, L;          // main tiles per workgroup (T / W) and the leftover tiles (T - q W)
  int cmax;          // shares per (leftover tile, XCD) at most
  void* partials;    // (kXcds + 1) * (q W + L cmax) partial tiles of the kernel's type
  double *G0, *gv0, *G1, *gv1;
  int64_t ldg;
  // rectangular products X^T J Y: A is X (n columns), Y has ny columns,
  // tiles run over mt x nt (tile = ti + mt tj), and the reduction writes
  // G0 = part 0 - part 1 (rows [0, p) minus rows [p, M))
  int mt, ny;
  const void* Y;
  int64_t ldy;
  // rectangular epilogue: C = alpha (part 0 - part 1) + beta C0 on columns j
  // with active[j] (or all when active is null); other columns get keep[:, j]
  // (or are left as they are when keep is null), and a tile whose columns are
  // all inactive is not computed
  double alpha, beta;
  const double* C0;
  int64_t ldc0;
  const int* active;
  const double* keep;
  int64_t ldkeep;
};

__device__ __host__ inline void pers_range(int64_t M, int x, int64_t& r0, int64_t& r1) {
  r0 = (M * x / kXcds) / kPersAlign * kPersAlign;
  r1 = x == kXcds - 1 ? M : (M * (x + 1) / kXcds) / kPersAlign * kPersAlign;
}
// Partial-tile block of XCD range x for `part`: the range itself, except the
// part-1 shares of the one range that holds rows on both sides of p, which
// go to block kXcds.
__device__ __host__ inline int pers_vx(int x, int part, int64_t r0, int64_t r1, int64_t p) {
  return (part == 1 && r0 < p && p < r1) ? kXcds : x;
}
// first workgroup (of W) whose share of TS stages contains stage u
__device__ __host__ inline int pers_first(int64_t u, int64_t TS, int W) {
  return (int)(((u + 1) * W - 1) / TS);
}

// Partial-tile index of the share of main tile t (t < q W) in block vx, and
// of share c of leftover tile lt in block vx.
__device__ __host__ inline size_t pers_slot_main(int vx, int t, int q, int W) {
  return (size_t)vx * q * W + t;
}
__device__ __host__ inline size_t pers_slot_left(int vx, int lt, int c, int q, int W, int L, int cmax) {
  return (size_t)(kXcds + 1) * q * W + ((size_t)vx * L + lt) * cmax + c;
}

static __device__ const double g_zero16[16] = {0.0};

// Issue-priority balancing of the resident workgroups.  A SIMD's arbiter
// favours its older waves, so the workgroups of one XCD, left alone, drift
// apart as they walk the range (at 20000 x 1000, 48 stages in, the earliest
// workgroup was 60 us into the launch and the latest 208 us): the L2 then
// serves each stage to fewer of the tiles that read it (reads 3.2x A) and
// the launch ends on a tail of the late workgroups.  Every ep_len stages each
// wave counts its arrival on the counter of its (XCD, wave slot, epoch) and
// takes its rank among the XCD's W workgroups as its issue priority (the
// first quarter lowest, the last quarter highest).  Nothing waits on the
// counters: they reorder issue only, so the arithmetic and its order are
// unchanged.  The reduction kernel clears them for the next launch (they
// start at zero); a launch that finds them not cleared only loses the
// balancing.
constexpr int kPersEpochs = 64;
static __device__ unsigned g_pers_rank[kXcds * 4 * kPersEpochs];

// s_waitcnt with a vector-memory limit only (vmcnt low bits 3:0, high bits
// 15:14; expcnt 6:4 and lgkmcnt 11:8 left at their maxima)
#define ILS_WAIT_VM(N) __builtin_amdgcn_s_waitcnt(((N) & 0xF) | (((N) >> 4) << 14) | (0x7 << 4) | (0xF << 8))

// Stage geometry per element type: a 16-byte chunk holds RPC rows of a
// column, a stage RS rows = 8 chunks (16 rows of FP64, 32 of FP32), so a
// stage of one operand is 8 KB either way.
template <typename T>
struct PersGeo {
  static constexpr int RPC = 16 / (int)sizeof(T);
  static constexpr int RS = 8 * RPC;
};

__device__ inline int pers_swz(int s) { return (s >> 1) & 7; }

// (the whole-range launch runs up to one workgroup per tile, 2 per CU at the
// shapes it takes, so it may use the registers of 2 waves per SIMD)
template <typename T, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(R == kGramWhole ? 2 : kPersWpc)))
void k_gram_pers(GramPJob job) {
  // R: kind of product, fixed at compile time so each instance carries only
  // its own code (kGramTri: lower tiles of A^T A with an optional border
  // column, partial tiles; kGramRect: X^T J Y, partial tiles; kGramWhole:
  // X^T Y, one workgroup per tile over all rows, C written directly)
  constexpr bool rect = R != kGramTri, whole = R == kGramWhole;
  typedef typename Mma<T>::acc_t acc_t;
  constexpr int RPC = PersGeo<T>::RPC, RS = PersGeo<T>::RS;
  __shared__ __attribute__((aligned(16))) T L[2][2][64 * RS];  // [stage][operand][slot * RS + row]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int lr = lane & 15;
  // whole-range launch: one workgroup per tile over all rows, no partials
  const int x = whole ? 0 : (int)(blockIdx.x % kXcds), j = whole ? (int)blockIdx.x : (int)(blockIdx.x / kXcds);
  int64_t r0 = 0, r1 = job.M;
  if (!whole) pers_range(job.M, x, r0, r1);
  const int64_t S = (r1 - r0 + RS - 1) / RS;
  if (S == 0) return;
  const int64_t LS = (int64_t)job.L * S;
  // main tiles over the whole range, then this workgroup's leftover stages
  const int64_t u0 = (int64_t)j * LS / job.W, u1 = (int64_t)(j + 1) * LS / job.W;
  const T* A = (const T*)job.A;
  const T* vb = (const T*)job.vb;
  const T* Y = (const T*)job.Y;
  const int64_t lda = job.lda, ldy = job.ldy;
  const int n = job.n;
  // column `col` of operand op (0: the tile's rows, 1: its columns), or null
  // for a zero slot
  auto opcol = [&](int op, int col) -> const T* {
    if (rect && op == 1) return col < job.ny ? Y + (int64_t)col * ldy : nullptr;
    if (col < n) return A + (int64_t)col * lda;
    return (!rect && col == n) ? vb : nullptr;
  };

  // issue-priority balancing (see g_pers_rank): epochs of ep_len stages,
  // the same length for every workgroup of the XCD
  const int64_t ep_len = whole ? 0 : ((int64_t)job.q * S + LS / job.W) / kPersEpochs + 8;
  int64_t done = 0, mark = ep_len;
  int ep = 0;
  unsigned rank = 0;
  bool rank_pend = false;
  auto balance = [&]() {
    if (whole) return;
    if (rank_pend) {
      // the count issued one stage ago has returned (the stage wait covers it)
      const int pr = __builtin_amdgcn_readfirstlane((int)rank) * 4 / job.W;
      if (pr <= 0) __builtin_amdgcn_s_setprio(0);
      else if (pr == 1) __builtin_amdgcn_s_setprio(1);
      else if (pr == 2) __builtin_amdgcn_s_setprio(2);
      else __builtin_amdgcn_s_setprio(3);
      rank_pend = false;
    }
    if (++done == mark) {
      mark += ep_len;
      if (ep < kPersEpochs) {
        if (lane == 0)
          rank = __hip_atomic_fetch_add(&g_pers_rank[(x * 4 + w) * kPersEpochs + ep], 1u, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        rank_pend = true;
        ++ep;
      }
    }
  };

  int mi = 0;
  for (int64_t u = u0; mi < job.q || u < u1;) {
    int tile, c = 0;
    int64_t klo, khi;
    const bool main = mi < job.q;
    if (main) {
      tile = j + mi * job.W;
      klo = r0;
      khi = r1;
      ++mi;
    } else {
      const int lt = (int)(u / S);
      const int64_t send = u1 < (int64_t)(lt + 1) * S ? u1 : (int64_t)(lt + 1) * S;
      c = j - pers_first((int64_t)lt * S, LS, job.W);
      tile = job.q * job.W + lt;
      klo = r0 + (u - (int64_t)lt * S) * RS;
      khi = r0 + (send - (int64_t)lt * S) * RS < r1 ? r0 + (send - (int64_t)lt * S) * RS : r1;
      u = send;
    }
    int ti, tj;
    if (rect) {
      ti = tile % job.mt;
      tj = tile / job.mt;
      if (job.active) {
        const int col = tj * 64 + (t & 63);
        if (!__syncthreads_or(t < 64 && col < job.ny && job.active[col])) continue;
      }
    } else {
      tile_of(tile, ti, tj);
    }
    // a diagonal tile loads its one panel twice, as every other tile loads
    // two: its workgroup then walks the rows in step with the rest instead of
    // running ahead (fetch 545 -> 452 MB per launch at 20000 x 1000)
    for (int part = 0; part < 2; ++part) {
      const int64_t kbeg = part ? (klo > job.p ? klo : job.p) : klo;
      const int64_t kend = part ? khi : (khi < job.p ? khi : job.p);
      if (kbeg >= kend) continue;
      acc_t acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) acc[a][cc] = acc_t{};
      auto compute = [&](int buf) {
        const T* La = &L[buf][0][0];
        const T* Lb = &L[buf][1][0];
#pragma unroll
        for (int kk = 0; kk < RS; kk += 4) {
          const int kr = kk + (lane >> 4);
          T fa[2], fb[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const int sl = wr + a * 16 + lr;
            fa[a] = La[sl * RS + (((kr / RPC) ^ pers_swz(sl)) * RPC) + (kr % RPC)];
          }
#pragma unroll
          for (int cc = 0; cc < 2; ++cc) {
            const int sl = wc + cc * 16 + lr;
            fb[cc] = Lb[sl * RS + (((kr / RPC) ^ pers_swz(sl)) * RPC) + (kr % RPC)];
          }
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) acc[a][cc] = Mma<T>::run(fa[a], fb[cc], acc[a][cc]);
        }
      };
      // rows [ka, kb) of buffer 0 through registers (within one stage), the rest zero
      auto reg_stage = [&](int64_t ka, int64_t kb) {
        __syncthreads();
        for (int id = t; id < 2 * 64 * 8; id += 256) {
          const int op = id / (64 * 8), sl = (id / 8) % 64, qc = id % 8;
          const T* cp = opcol(op, (op ? tj : ti) * 64 + sl);
          T* d = &L[0][op][sl * RS + ((qc ^ pers_swz(sl)) * RPC)];
#pragma unroll
          for (int e = 0; e < RPC; ++e) {
            const int64_t r = ka + qc * RPC + e;
            d[e] = (cp && r < kb) ? cp[r] : (T)0;
          }
        }
        __syncthreads();
        compute(0);
      };
      int64_t ka = kbeg;
      if (ka % RPC) {  // first row off a 16-byte boundary: up to it through registers
        const int64_t kn = (ka / RPC + 1) * RPC < kend ? (ka / RPC + 1) * RPC : kend;
        reg_stage(ka, kn);
        ka = kn;
      }
      const int64_t nfull = (kend - ka) / RS;
      if (nfull > 0) {
        // this lane's sources: load i of operand op fills slots (2w + i) * 8 + lane / 8, chunk lane % 8
        const T* src[2][2];
        int64_t step[2][2];
#pragma unroll
        for (int op = 0; op < 2; ++op)
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const int sl = (2 * w + i) * 8 + (lane >> 3);
            const int sig = (lane & 7) ^ pers_swz(sl);
            const T* cp = opcol(op, (op ? tj : ti) * 64 + sl);
            if (cp) {
              src[op][i] = cp + ka + RPC * sig;
              step[op][i] = RS;
            } else {
              src[op][i] = (const T*)g_zero16 + RPC * sig;
              step[op][i] = 0;
            }
          }
        auto issue = [&](int64_t st, int buf) {
#pragma unroll
          for (int i = 0; i < 2; ++i)
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void*)(src[0][i] + st * step[0][i]),
                (__attribute__((address_space(3))) void*)&L[buf][0][(2 * w + i) * (1024 / (int)sizeof(T))], 16, 0, 0);
#pragma unroll
          for (int i = 0; i < 2; ++i)
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void*)(src[1][i] + st * step[1][i]),
                (__attribute__((address_space(3))) void*)&L[buf][1][(2 * w + i) * (1024 / (int)sizeof(T))], 16, 0,
                0);
        };
        __syncthreads();  // buffer 0 may still be read by a register stage
        issue(0, 0);
        for (int64_t st = 0; st < nfull; ++st) {
          // this wave's loads of stage st have landed; after the barrier every
          // wave's have, and every wave is done reading the other buffer
          ILS_WAIT_VM(0);
          __asm__ __volatile__("" ::: "memory");
          __builtin_amdgcn_s_barrier();
          __asm__ __volatile__("" ::: "memory");
          if (st + 1 < nfull) issue(st + 1, (int)((st + 1) & 1));
          balance();
          compute((int)(st & 1));
        }
      }
      const int64_t kt = ka + nfull * RS;
      if (kt < kend) reg_stage(kt, kend);
      if (whole) {
        // the tile's final value with the rectangular epilogue
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
          const int jj = tj * 64 + wc + cc * 16 + lr;
          if (jj >= job.ny) continue;
          const bool live = !job.active || job.active[jj];
          if (!live && !job.keep) continue;
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int i = ti * 64 + wr + a * 16 + Mma<T>::row(lane, v);
              if (i >= n) continue;
              double val;
              if (live) {
                val = job.alpha * (double)acc[a][cc][v];
                if (job.beta != 0.0) val += job.beta * job.C0[i + (int64_t)jj * job.ldc0];
              } else {
                val = job.keep[i + (int64_t)jj * job.ldkeep];
              }
              job.G0[i + (int64_t)jj * job.ldg] = val;
            }
        }
      } else {
        const int vx = pers_vx(x, part, r0, r1, job.p);
        T* P = (T*)job.partials + (main ? pers_slot_main(vx, tile, job.q, job.W)
                                        : pers_slot_left(vx, tile - job.q * job.W, c, job.q, job.W, job.L,
                                                         job.cmax)) *
                                      4096;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int cc = 0; cc < 2; ++cc)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = wr + a * 16 + Mma<T>::row(lane, v);
              const int col = wc + cc * 16 + lr;
              P[row * 64 + col] = acc[a][cc][v];
            }
      }
      __syncthreads();  // LDS free for the next share
    }
  }
}

// Per (tile, part): the shares of XCD 0..7 in row order (share index c within
// an XCD follows the rows).  Wave 0 lists them, one (XCD, c) pair per lane in
// that order, compacted by ballot; then every thread adds its element.
template <typename T, int R>
__global__ __launch_bounds__(256) void k_gram_pers_fin(GramPJob job) {
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int e = threadIdx.x; e < kXcds * 4 * kPersEpochs; e += blockDim.x) g_pers_rank[e] = 0u;
  constexpr bool rect = R == kGramRect;
  constexpr int RS = PersGeo<T>::RS;
  __shared__ int slots[2][kXcds * kPersMaxShares];
  __shared__ int nsl[2];
  // rectangular product: one block per tile adds part 0 and subtracts part 1
  const int part = rect ? 0 : (int)blockIdx.y / job.T, tile = (int)blockIdx.y % job.T;
  const int nlists = rect ? 2 : 1;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    for (int li = 0; li < nlists; ++li) {
      const int pt = rect ? li : part;
      const int64_t lo = pt ? job.p : 0, hi = pt ? job.M : job.p;
      const bool main = tile < job.q * job.W;
      const int lt = tile - job.q * job.W;
      const int per = main ? 1 : job.cmax;  // pairs (XCD, share) per XCD
      int base = 0;
      for (int p0 = 0; p0 < kXcds * per; p0 += 64) {
        const int pair = p0 + lane;
        const int x = pair / per, c = pair % per;
        int slot = -1;
        if (x < kXcds) {
          int64_t r0, r1;
          pers_range(job.M, x, r0, r1);
          const int64_t S = (r1 - r0 + RS - 1) / RS;
          int64_t klo = r0, khi = r1;
          bool ok = S > 0;
          if (ok && !main) {
            const int64_t LS = (int64_t)job.L * S;
            const int j = pers_first((int64_t)lt * S, LS, job.W) + c;
            ok = j < job.W;
            if (ok) {
              const int64_t u0 = (int64_t)j * LS / job.W, u1 = (int64_t)(j + 1) * LS / job.W;
              const int64_t a = u0 > (int64_t)lt * S ? u0 : (int64_t)lt * S;
              const int64_t b = u1 < (int64_t)(lt + 1) * S ? u1 : (int64_t)(lt + 1) * S;
              ok = a < b;
              klo = r0 + (a - (int64_t)lt * S) * RS;
              khi = r0 + (b - (int64_t)lt * S) * RS;
              if (khi > r1) khi = r1;
            }
          }
          if (ok && (klo > lo ? klo : lo) < (khi < hi ? khi : hi)) {
            const int vx = pers_vx(x, pt, r0, r1, job.p);
            slot = (int)(main ? pers_slot_main(vx, tile, job.q, job.W)
                              : pers_slot_left(vx, lt, c, job.q, job.W, job.L, job.cmax));
          }
        }
        const uint64_t m = __ballot(slot >= 0);
        if (slot >= 0) slots[li][base + __popcll(m & ((1ull << lane) - 1))] = slot;
        base += __popcll(m);
      }
      if (lane == 0) nsl[li] = base;
    }
  }
  __syncthreads();
  int ti, tj;
  if (rect) {
    ti = tile % job.mt;
    tj = tile / job.mt;
  } else {
    tile_of(tile, ti, tj);
  }
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int row = e / 64, col = e % 64;
  const int i = ti * 64 + row, jj = tj * 64 + col;
  if (rect) {
    if (i >= job.n || jj >= job.ny) return;
    if (job.active && !job.active[jj]) {
      if (job.keep) job.G0[i + (int64_t)jj * job.ldg] = job.keep[i + (int64_t)jj * job.ldkeep];
      return;
    }
  } else if (i >= job.nc || jj >= job.nc || (ti == tj && row < col) || (i == job.n && jj == job.n)) {
    return;
  }
  const T* partials = (const T*)job.partials;
  auto add_list = [&](int li) {
    const int cnt = nsl[li];
    double sacc = 0.0;
    int q = 0;
    for (; q + 8 <= cnt; q += 8) {
      double v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = (double)partials[(size_t)slots[li][q + k] * 4096 + e];
#pragma unroll
      for (int k = 0; k < 8; ++k) sacc += v[k];
    }
    for (; q < cnt; ++q) sacc += (double)partials[(size_t)slots[li][q] * 4096 + e];
    return sacc;
  };
  if (rect) {
    double v = job.alpha * (add_list(0) - add_list(1));
    if (job.beta != 0.0) v += job.beta * job.C0[i + (int64_t)jj * job.ldc0];
    job.G0[i + (int64_t)jj * job.ldg] = v;
    return;
  }
  const double sacc = add_list(0);
  double* G = part ? job.G1 : job.G0;
  double* gv = part ? job.gv1 : job.gv0;
  if (i == job.n) {
    gv[jj] = sacc;
    return;
  }
  G[i + (int64_t)jj * job.ldg] = sacc;
  G[jj + (int64_t)i * job.ldg] = sacc;
}

static int device_cus() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev < 0 || dev >= 64) return 256;
  if (!cache[dev]) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < kXcds) c = 256;
    cache[dev] = c;
  }
  return cache[dev];
}

// Largest number of workgroups sharing one leftover tile within one XCD range
// (stages of RS rows).
static int pers_cmax(int64_t M, int L, int W, int RS) {
  int cm = 1;
  for (int x = 0; x < kXcds && L > 0; ++x) {
    int64_t r0, r1;
    pers_range(M, x, r0, r1);
    const int64_t S = (r1 - r0 + RS - 1) / RS;
    const int64_t LS = (int64_t)L * S;
    if (LS == 0) continue;
    for (int j = 0; j < W; ++j) {
      const int64_t u0 = (int64_t)j * LS / W, u1 = (int64_t)(j + 1) * LS / W;
      for (int64_t u = u0; u < u1;) {
        const int lt = (int)(u / S);
        cm = std::max(cm, j - pers_first((int64_t)lt * S, LS, W) + 1);
        u = std::min(u1, (int64_t)(lt + 1) * S);
      }
    }
  }
  return cm;
}

struct PersShape {
  int T, W, q, L, cmax;
};
static PersShape pers_shape_t(int T, int64_t M, int RS);
static PersShape pers_shape(int64_t nc, int64_t M, int RS) {
  const int nt = (int)((nc + 63) / 64);
  return pers_shape_t(nt * (nt + 1) / 2, M, RS);
}
// The plan for T tiles over M rows in stages of RS rows.
static PersShape pers_shape_t(int T, int64_t M, int RS) {
  static std::mutex mu;
  static std::map<std::tuple<int64_t, int64_t, int, int>, int> cache;
  PersShape sh;
  sh.T = T;
  sh.W = kPersWpc * (device_cus() / kXcds);
  sh.q = sh.T / sh.W;
  sh.L = sh.T - sh.q * sh.W;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple((int64_t)T, M, sh.W, RS);
  auto it = cache.find(key);
  if (it == cache.end()) {
    if (cache.size() > 256) cache.clear();
    it = cache.emplace(key, pers_cmax(M, sh.L, sh.W, RS)).first;
  }
  sh.cmax = it->second;
  return sh;
}

// Partial tiles in doubles (either element type's tiles fit).
static size_t pers_partials(int64_t nc, int64_t M) {
  size_t s = 0;
  for (int RS : {PersGeo<double>::RS, PersGeo<float>::RS}) {
    const PersShape sh = pers_shape(nc, M, RS);
    s = std::max(s, ((size_t)(kXcds + 1) * ((size_t)sh.q * sh.W + (size_t)sh.L * sh.cmax)) * 4096);
  }
  return s;
}

// 16-byte aligned columns: the base and the border column on 16 bytes, lda a
// multiple of 16 / sizeof(T).
template <typename T>
static bool pers_aligned(const T* A, int64_t lda, const T* vb) {
  return ((uintptr_t)A & 15) == 0 && (lda % (16 / (int64_t)sizeof(T))) == 0 && (!vb || ((uintptr_t)vb & 15) == 0);
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
  c.kind = kGramSplitK;
  return c;
}

// Without a table entry: the persistent kernel (FP32 from a copy of the
// rows) for products with enough columns and rows to give every resident workgroup several stages,
// and few enough tiles that splitting the rows per XCD stays cheap.
static GramCfg auto_cfg(int precision, int64_t n, int64_t K) {
  if (n >= 192 && K >= 2048) {
    const int nt = (int)((n + 1 + 63) / 64);
    if (nt * (nt + 1) / 2 <= 2 * kPersWpc * (device_cus() / kXcds)) return GramCfg{64, kPersWpc, kGramPersistent};
  }
  return gram_default_cfg(n);
}

GramCfg gram_cfg(int precision, int64_t n, int64_t K) {
  {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    auto it = g_cfg.find(cfg_key(precision, n, K));
    if (it != g_cfg.end()) return it->second;
  }
  return auto_cfg(precision, n, K);
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

// The split-K configuration behind cfg (a persistent entry falls back to the
// default split-K launch where the persistent kernel does not apply).
static GramCfg splitk_of(GramCfg c, int64_t n) { return c.kind == kGramSplitK ? c : gram_default_cfg(n); }

static size_t plan_size(int64_t n, int64_t K, GramCfg c) {
  int tm, ntiles, nsplit;
  int64_t klen;
  gram_plan_cfg(n, K, splitk_of(c, n), tm, ntiles, nsplit, klen);
  size_t sz = (size_t)ntiles * nsplit * tm * tm;
  if (c.kind == kGramPersistent) sz = std::max(sz, pers_partials(n, K));
  return sz;
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
  const GramCfg c = gram_cfg(ILS_PREC_FP64, n, K0);
  gram_plan_cfg(n + 1, K0, splitk_of(c, n), tm, ntiles, ns0, kl0);
  second_plan(K1, kl0, ns1, kl1);
  size_t sz = std::max((size_t)ntiles * (ns0 + ns1) * tm * tm, gram_partials_size(n, K0));
  if (c.kind == kGramPersistent) sz = std::max(sz, pers_partials(n + 1, K0 + std::max<int64_t>(K1, 0)));
  return sz;
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
  if (std::is_same<T, double>::value && cfg.kind == kGramPersistent && pers_aligned<double>(A, lda, vb) &&
      (K1 < 0 || (A1 == A + K && (vb ? vb1 == vb + K : vb1 == nullptr)))) {
    GramPJob pj = {};
    pj.A = A;
    pj.lda = lda;
    pj.vb = vb;
    pj.M = K + (K1 > 0 ? K1 : 0);
    pj.p = K;
    pj.n = (int)n;
    pj.nc = (int)n + (vb ? 1 : 0);
    const PersShape sh = pers_shape(pj.nc, pj.M, PersGeo<double>::RS);
    pj.T = sh.T;
    pj.W = sh.W;
    pj.q = sh.q;
    pj.L = sh.L;
    pj.cmax = sh.cmax;
    if (sh.cmax <= kPersMaxShares) {
      pj.partials = (double*)partials;
      pj.G0 = G;
      pj.gv0 = gv;
      pj.G1 = G1;
      pj.gv1 = gv1;
      pj.ldg = ldg;
      hipLaunchKernelGGL((k_gram_pers<double, kGramTri>), dim3(kXcds * sh.W), dim3(256), 0, s, pj);
      if (mid) (void)hipEventRecord(mid, s);
      hipLaunchKernelGGL((k_gram_pers_fin<double, kGramTri>), dim3(64 * 64 / 256, sh.T * (K1 >= 0 ? 2 : 1)), dim3(256), 0, s,
                         pj);
      return;
    }
  }
  cfg = splitk_of(cfg, n);
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

// A^T A of an FP32 matrix (K x n, column-major, ldaf, 16-byte aligned
// columns) with the persistent kernel.
static void gram_f32_pers(hipStream_t s, int64_t K, int64_t n, const float* Af, int64_t ldaf, float* partials,
                          double* G, int64_t ldg, hipEvent_t mid) {
  GramPJob pj = {};
  pj.A = Af;
  pj.lda = ldaf;
  pj.vb = nullptr;
  pj.M = K;
  pj.p = K;
  pj.n = (int)n;
  pj.nc = (int)n;
  const PersShape sh = pers_shape(n, K, PersGeo<float>::RS);
  pj.T = sh.T;
  pj.W = sh.W;
  pj.q = sh.q;
  pj.L = sh.L;
  pj.cmax = sh.cmax;
  pj.partials = partials;
  pj.G0 = G;
  pj.gv0 = nullptr;
  pj.G1 = nullptr;
  pj.gv1 = nullptr;
  pj.ldg = ldg;
  hipLaunchKernelGGL((k_gram_pers<float, kGramTri>), dim3(kXcds * sh.W), dim3(256), 0, s, pj);
  if (mid) (void)hipEventRecord(mid, s);
  hipLaunchKernelGGL((k_gram_pers_fin<float, kGramTri>), dim3(64 * 64 / 256, sh.T), dim3(256), 0, s, pj);
}

// The product of GemmTnArgs, C = alpha X^T S Y + beta C0 (S = diag(I_kneg,
// -I_{K-kneg}); X: K x M, Y: K x N, column-major, K contiguous; optional
// column mask and keep) on the persistent kernel: 64 x 64 tiles of C over
// the same per-XCD row ranges, the two signs as the kernel's two row parts,
// subtracted in the reduction, which also applies the epilogue.  False
// (nothing queued) when the operands are not 16-byte aligned with even
// leading dimensions, the plan needs more shares per tile than the reduction
// lists, or `partials` is smaller than gemm_tn_pers_partials.
static int rect_tiles(int64_t M, int64_t N) { return (int)(((M + 63) / 64) * ((N + 63) / 64)); }
// longest contraction the whole-range launch takes (above it, the row split
// over XCDs keeps each tile's stages shared in one L2)
constexpr int64_t kWholeMaxK = 4096;

size_t gemm_tn_pers_partials(int64_t K, int64_t M, int64_t N) {
  const PersShape sh = pers_shape_t(rect_tiles(M, N), K, PersGeo<double>::RS);
  return ((size_t)(kXcds + 1) * ((size_t)sh.q * sh.W + (size_t)sh.L * sh.cmax)) * 4096;
}

bool launch_gemm_tn_pers(hipStream_t s, const GemmTnArgs& g, double* partials, size_t partial_doubles) {
  const int64_t K = g.K, M = g.M, N = g.N;
  if (K < 1 || M < 1 || N < 1 || !pers_aligned<double>(g.X, g.ldx, nullptr) ||
      !pers_aligned<double>(g.Y, g.ldy, nullptr))
    return false;
  const int T = rect_tiles(M, N);
  if (g.kneg >= K && K <= kWholeMaxK && T <= kPersWpc * device_cus()) {
    // short contraction, one sign: a workgroup per tile walks all K rows and
    // writes its tile of C (no row split over XCDs, no partials)
    GramPJob pj = {};
    pj.A = g.X;
    pj.lda = g.ldx;
    pj.M = K;
    pj.p = K;
    pj.n = (int)M;
    pj.nc = (int)M;
    pj.T = T;
    pj.W = T;
    pj.q = 1;
    pj.L = 0;
    pj.cmax = 1;
    pj.G0 = g.C;
    pj.ldg = g.ldc;
    pj.mt = (int)((M + 63) / 64);
    pj.ny = (int)N;
    pj.Y = g.Y;
    pj.ldy = g.ldy;
    pj.alpha = g.alpha;
    pj.beta = g.beta;
    pj.C0 = g.C0;
    pj.ldc0 = g.ldc0;
    pj.active = g.active;
    pj.keep = g.keep;
    pj.ldkeep = g.ldkeep;
    hipLaunchKernelGGL((k_gram_pers<double, kGramWhole>), dim3(T), dim3(256), 0, s, pj);
    return true;
  }
  const PersShape sh = pers_shape_t(T, K, PersGeo<double>::RS);
  if (sh.cmax > kPersMaxShares || gemm_tn_pers_partials(K, M, N) > partial_doubles) return false;
  GramPJob pj = {};
  pj.A = g.X;
  pj.lda = g.ldx;
  pj.vb = nullptr;
  pj.M = K;
  pj.p = g.kneg < K ? g.kneg : K;
  pj.n = (int)M;
  pj.nc = (int)M;
  pj.T = sh.T;
  pj.W = sh.W;
  pj.q = sh.q;
  pj.L = sh.L;
  pj.cmax = sh.cmax;
  pj.partials = partials;
  pj.G0 = g.C;
  pj.ldg = g.ldc;
  pj.mt = (int)((M + 63) / 64);
  pj.ny = (int)N;
  pj.Y = g.Y;
  pj.ldy = g.ldy;
  pj.alpha = g.alpha;
  pj.beta = g.beta;
  pj.C0 = g.C0;
  pj.ldc0 = g.ldc0;
  pj.active = g.active;
  pj.keep = g.keep;
  pj.ldkeep = g.ldkeep;
  hipLaunchKernelGGL((k_gram_pers<double, kGramRect>), dim3(kXcds * sh.W), dim3(256), 0, s, pj);
  hipLaunchKernelGGL((k_gram_pers_fin<double, kGramRect>), dim3(64 * 64 / 256, sh.T), dim3(256), 0, s, pj);
  return true;
}

// Column-major FP32 copy of rows [0, K) of A with leading dimension ldaf.
__global__ void k_copy_f32(int64_t K, int64_t n, const double* __restrict__ A, int64_t lda, float* __restrict__ Af,
                           int64_t ldaf) {
  for (int64_t c = blockIdx.y; c < n; c += gridDim.y)
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < K; i += (int64_t)gridDim.x * 256)
      Af[i + c * ldaf] = (float)A[i + c * lda];
}

int64_t gram_f32_copy_ld(int64_t K) { return (K + 3) / 4 * 4; }

// The FP32 product through a copy: the copy must be 16-byte aligned (it is,
// with the leading dimension above, from any allocation) and the shape within
// the shares the reduction lists.
static bool f32_copy_fits(int64_t n, int64_t K, const float* Af) {
  return Af && ((uintptr_t)Af & 15) == 0 && pers_shape(n, K, PersGeo<float>::RS).cmax <= kPersMaxShares;
}

static void gram_f32_via_copy(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda, float* Af,
                              float* partials, double* G, int64_t ldg, hipEvent_t mid) {
  const int64_t ldaf = gram_f32_copy_ld(K);
  const int64_t bx = std::min<int64_t>(std::max<int64_t>((K + 255) / 256, 1), 64);
  const int64_t by = std::min<int64_t>(n, 65535);
  hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)bx, (unsigned)by), dim3(256), 0, s, K, n, A, lda, Af, ldaf);
  gram_f32_pers(s, K, n, Af, ldaf, partials, G, ldg, mid);
}

void launch_gram_cfg(hipStream_t s, int precision, int64_t K, int64_t n, const double* A, int64_t lda,
                     void* partials, double* G, int64_t ldg, GramCfg cfg, float* a1f) {
  if (precision == ILS_PREC_MIXED && cfg.kind == kGramPersistent && f32_copy_fits(n, K, a1f)) {
    gram_f32_via_copy(s, K, n, A, lda, a1f, (float*)partials, G, ldg, nullptr);
    return;
  }
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


bool gram_f32_uses_copy(int64_t n, int64_t K) {
  return gram_cfg(ILS_PREC_MIXED, n, K).kind == kGramPersistent &&
         pers_shape(n, K, PersGeo<float>::RS).cmax <= kPersMaxShares;
}

void launch_gram_f32_on_copy(hipStream_t s, int64_t K, int64_t n, const float* Af, float* partials, double* G,
                             int64_t ldg, hipEvent_t mid) {
  gram_f32_pers(s, K, n, Af, gram_f32_copy_ld(K), partials, G, ldg, mid);
}

void launch_gram_f32_copy(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda, float* Af,
                          float* partials, double* G, int64_t ldg, hipEvent_t mid) {
  if (f32_copy_fits(n, K, Af))
    gram_f32_via_copy(s, K, n, A, lda, Af, partials, G, ldg, mid);
  else
    launch_gram_f32(s, K, n, A, lda, partials, G, ldg, mid);
}

void launch_gram_f32(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda,
                     float* partials, double* G, int64_t ldg, hipEvent_t mid) {
  gram_run<float>(s, K, n, A, lda, nullptr, partials, G, ldg, nullptr, mid, gram_cfg(ILS_PREC_MIXED, n, K));
}

}  // namespace ils
