// ils_common.hpp -- internal declarations shared by the gfx950 kernels and the
// host runtime of the ILS splitting solver.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ils.h"

namespace ils {

constexpr int kWave = 64;  // CDNA wavefront width

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Status bits raised on the device; the host maps them to ils_status.
enum : int {
  kBitNonfinite = 1,  // NaN/Inf in A or b
  kBitNotSpd = 2,     // a Gauss-Jordan pivot block is not positive definite
  kBitStall = 4,      // a dataflow kernel's bounded wait ran out (never expected)
};

// Device-side state of an outer loop (one per handle).
struct LoopState {
  int done;           // 0 running, else finished (SP step: deciding launch + 1)
  int status;         // ils_status of the finished loop
  int64_t iters;      // outer updates performed when done
  double metric;      // stop quantity at the final iterate
  int bits;           // kBit* flags raised by setup kernels
  int64_t inner_total;// randomized methods: inner steps taken
  int inner_done;     // randomized methods: inner stop test met
  unsigned int arrive2;// last-block counter of the inner test
  int64_t steps;      // SP-SCD: inner steps of the current outer step
  double scal[8];     // small device scalars: 0 ||A^T J b||^2, 1 ||x_ref||^2,
                      // 2 ||inner target||^2, 7 relative error
  int nactive;        // multi-right-hand-side solve: columns still iterating
  unsigned int arrive3;// last-block counter of the blocked RK-RGS steps
  int resid_skip;     // SP correction form: the last residual pass was skipped
};

// Pointers loaded from memory or passed to out-of-line functions are generic,
// and accesses through them compile to flat instructions, which count against
// both the vector-memory and the LDS wait counters (a wait for an LDS read then
// also waits for every load in flight).  Recasting a pointer known to address
// device memory to the global address space gives global_* instructions.
template <typename T>
__device__ inline __attribute__((address_space(1))) T* glb(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// ---------------------------------------------------------------- reductions
// Sum over the 64 lanes of a wavefront, every lane of which must be active;
// every lane gets the same bits.  DPP moves pair the lanes: within each row
// of 16, lane ^ 1, lane ^ 2, then the mirrors within 8 and within 16 lanes
// (each pair adds the same two values, so a row's lanes agree); then lane
// 15 of rows 0 and 2 is added into rows 1 and 3, and lane 31 into rows 2
// and 3, so lane 63 holds the total, which is read back to all lanes.  The
// order is fixed, so results are reproducible run to run; a row of 64-bit
// moves and adds costs a small part of the six LDS permutes of a shuffle
// butterfly.
// Sum over each row of 16 lanes, every lane of the row getting the same bits.
template <typename T>
__device__ inline T row16_sum(T v) {
  v += __builtin_amdgcn_update_dpp((T)0, v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  v += __builtin_amdgcn_update_dpp((T)0, v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  v += __builtin_amdgcn_update_dpp((T)0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += __builtin_amdgcn_update_dpp((T)0, v, 0x140, 0xF, 0xF, false);  // row_mirror
  return v;
}
// The value of lane l ^ 16 and of lane l ^ 32 (all lanes active), by the
// gfx950 permlane swaps instead of an LDS permute: with both operands the
// same register, the swap of rows 1, 3 with rows 0, 2 (of lanes 32-63 with
// lanes 0-31) leaves the partner's value in the first result on odd rows
// (upper lanes) and in the second on even rows (lower lanes).
__device__ inline double lane_xor16(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const bool odd = (threadIdx.x >> 4) & 1;
  return __hiloint2double(odd ? b[0] : b[1], odd ? a[0] : a[1]);
}
__device__ inline double lane_xor32(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const bool upper = (threadIdx.x >> 5) & 1;
  return __hiloint2double(upper ? b[0] : b[1], upper ? a[0] : a[1]);
}

template <typename T>
__device__ inline T wave_sum_dpp(T v) {
  v = row16_sum(v);
  v += __builtin_amdgcn_update_dpp((T)0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
  v += __builtin_amdgcn_update_dpp((T)0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
  return v;
}
__device__ inline double wave_sum(double v) {
  v = wave_sum_dpp(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), kWave - 1);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), kWave - 1);
  return __hiloint2double(hi, lo);
}
__device__ inline float wave_sum(float v) {
  v = wave_sum_dpp(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kWave - 1));
}

// Sum over a workgroup of NT threads; every thread gets the result.  `red`
// is LDS scratch of NT/64 doubles; the caller alternates two scratch areas
// between consecutive calls (or separates them by a barrier).
template <int NT, typename T>
__device__ inline T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int i = 1; i < NT / kWave; ++i) s += red[i];
  return s;
}

// ---------------------------------------------------------------- PRNG
// Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ inline void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                     uint64_t k0, uint64_t k1, uint64_t out[4]) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B97F4A7C15ull;
      k1 += 0xBB67AE8584CAA73Bull;
    }
    const uint64_t lo0 = 0xD2E7470EE14C6C93ull * c0, hi0 = __umul64hi(0xD2E7470EE14C6C93ull, c0);
    const uint64_t lo1 = 0xCA5A826395121157ull * c2, hi1 = __umul64hi(0xCA5A826395121157ull, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// SplitMix64 output function (Steele, Lea, Flood, OOPSLA'14).
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline double u01(uint64_t v) { return (double)(v >> 11) * (1.0 / 9007199254740992.0); }
__device__ inline int64_t uniform_below(uint64_t v, int64_t n) { return (int64_t)__umul64hi(v, (uint64_t)n); }

// Method tags in the Philox key: (seed, tag).
constexpr uint64_t kTagRk = 0x524B524753ull;
constexpr uint64_t kTagScd = 0x534344ull;

// ---------------------------------------------------------------- launchers
// Dense building blocks (k_dense.hip).
void launch_colpass(hipStream_t s, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                    const double* b, double* g, double* cn, int* bits, float* a1f = nullptr, int64_t ldaf = 0);
// r = A^T J (b - A x); t is residual_scratch(m, n) doubles of scratch (t = b - A x
// in the first m).  Skipped when *done != 0.
void launch_border_combine(hipStream_t s, int64_t n, double* g, const double* g2, const double* G1,
                           const double* G2, int64_t ldg, double* gcol, int* bits);
// Residual launch choice: kResidAuto takes the one-pass kernel for n <= 1024
// with `wgs` workgroups, kResidTwoPass always the row pass + column pass.
// The table (autotuner) supplies it per (log2 n, log2 m); the scratch a
// caller allocates with residual_scratch covers the table's and the default
// choice.
enum { kResidAuto = 0, kResidTwoPass = 1 };
constexpr int kResidDefaultWgs = 256;
struct ResidCfg {
  int path = kResidAuto;
  int wgs = kResidDefaultWgs;
};
ResidCfg residual_cfg(int64_t n, int64_t m);
size_t residual_scratch(int64_t m, int64_t n);
size_t residual_scratch_cfg(int64_t m, int64_t n, ResidCfg c);
// SP step geometry: rows per workgroup (one wave each) and threads
constexpr int kSpRows = 4;
constexpr int kSpThreads = kSpRows * kWave;

// The SP step's stop quantity from the summed partials: relative error
// against x_ref, or RR (Sec. 5).  One definition for every kernel that takes
// the stopping test, so all reach the same decision bit for bit.
__device__ inline double sp_metric(double tot, int stop_rule, const double* scal) {
  if (stop_rule == ILS_STOP_XREF) return sqrt(tot) / sqrt(scal[1]);
  if (stop_rule == ILS_STOP_RR) return tot / scal[0];
  return 0.0;
}

// The stopping tests that SP step launches will take, repeated by a kernel
// queued before them (the same partials added in the same order): a
// correction-form residual for an iterate the loop will not use is skipped.
// Test 1 is launch kk + 1's test on x_kk (partials of x_kk's metric, flags of
// x_{kk+1}); test 2 (part_next non-null) the end of the loop at x_kk + 1 by
// its metric or the step limit alone.  part == null: no test.
struct SpStopCheck {
  const double* part;       // metric partials of x_kk (nblk entries)
  const int* pbad;          // non-finite flags of x_{kk+1} (nblk entries)
  const double* part_next;  // metric partials of x_{kk+1}, or null
  int nblk;
  int stop_rule;
  double tol;
  int64_t kk, max_outer;
  const double* scal;  // LoopState::scal
  int* skip;           // set to whether the test ended the loop (read by the follow-up kernel)
};
void launch_residual(hipStream_t s, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                     const double* b, const double* x, double* t, double* r, const int* done,
                     const SpStopCheck* chk = nullptr);
void launch_residual_cfg(hipStream_t s, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                         const double* b, const double* x, double* t, double* r, const int* done, ResidCfg c,
                         const SpStopCheck* chk = nullptr);
// Gram of rows [0, K) of A (A already offset to the first row).  `partials`
// must hold gram_partials_size(n, K) doubles.
size_t gram_partials_size(int64_t n, int64_t K);
// With a border column vb (K entries, may be null) the product of the
// bordered matrix [A vb] also yields A^T vb, written to gv (n entries).
void launch_gram_f64(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda,
                     double* partials, double* G, int64_t ldg, hipEvent_t mid = nullptr,
                     const double* vb = nullptr, double* gv = nullptr);
void launch_gram_f32(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda,
                     float* partials, double* G, int64_t ldg, hipEvent_t mid = nullptr);
// FP32 Gram through an FP32 copy of the K rows (Af: gram_f32_copy_ld(K) x n
// floats of scratch, 16-byte aligned), formed first; taken when the launch
// table's mixed entry for (n, K) is the persistent kind and the shape suits
// it (gram_f32_uses_copy), which then reads half the bytes of the FP64 rows.
int64_t gram_f32_copy_ld(int64_t K);
bool gram_f32_uses_copy(int64_t n, int64_t K);
void launch_gram_f32_copy(hipStream_t s, int64_t K, int64_t n, const double* A, int64_t lda, float* Af,
                          float* partials, double* G, int64_t ldg, hipEvent_t mid = nullptr);
// The same product when Af already holds the copy (written by the column
// pass): only the persistent kernel and its reduction are queued.
void launch_gram_f32_on_copy(hipStream_t s, int64_t K, int64_t n, const float* Af, float* partials, double* G,
                             int64_t ldg, hipEvent_t mid = nullptr);
// Both bordered products [A0 vb0]^T [A0 vb0] and [A1 vb1]^T [A1 vb1] in one
// launch pair (FP64, part 0's configuration); `partials` must hold
// gram2_partials_size(n, K0, K1) doubles.
size_t gram2_partials_size(int64_t n, int64_t K0, int64_t K1);
void launch_gram2_f64(hipStream_t s, int64_t n, int64_t lda, int64_t ldg, double* partials, hipEvent_t mid,
                      int64_t K0, const double* A0, const double* vb0, double* G0, double* gv0,
                      int64_t K1, const double* A1, const double* vb1, double* G1, double* gv1);
// Gram launch configuration and the tuning table consulted by
// launch_gram_f64/f32.  kind kGramSplitK: tile edge 64 or 128 and the
// workgroups aimed at (which set the K-split); kind kGramPersistent (FP64):
// the resident 64-tile kernel with direct global-to-LDS loads (tile 64,
// workgroups = per CU).
enum { kGramSplitK = 0, kGramPersistent = 1 };
constexpr int kGramPersistentWpc = 4;  // resident workgroups per CU of the persistent kind
struct GramCfg {
  int tile;
  int workgroups;
  int kind = kGramSplitK;
};
struct GramCfgEntry {
  int precision, n_bucket, k_bucket;
  GramCfg cfg;
};
GramCfg gram_default_cfg(int64_t n);
GramCfg gram_cfg(int precision, int64_t n, int64_t K);
void gram_set_cfg(int precision, int64_t n, int64_t K, GramCfg c);
void gram_set_cfg_bucket(int precision, int n_bucket, int k_bucket, GramCfg c);
void gram_clear_cfg();
size_t gram_partials_size_cfg(int64_t n, int64_t K, GramCfg c);
void launch_gram_cfg(hipStream_t s, int precision, int64_t K, int64_t n, const double* A, int64_t lda,
                     void* partials, double* G, int64_t ldg, GramCfg cfg, float* a1f = nullptr);
void launch_norm2(hipStream_t s, int64_t n, const double* v, double* out);
// LoopState zeroed, and ||x_ref||^2 into its scal[1] when x_ref is given.
void launch_state_reset(hipStream_t s, LoopState* st, int64_t n, const double* x_ref);
void launch_transpose(hipStream_t s, int64_t n, int64_t ncol, const double* X, int64_t ldx,
                      double* Y, int64_t ldy);
void launch_copy_cols(hipStream_t s, int64_t n, int64_t ncol, const double* X, int64_t ldx,
                      double* Y, int64_t ldy);
void launch_fill_vec(hipStream_t s, int64_t n, const double* src, double* dst);
void launch_eye(hipStream_t s, int64_t n, double* Y, int64_t ldy);
void launch_diag_screen(hipStream_t s, int64_t n, const double* G1, const double* G2, int64_t ldg, int* bits);
void launch_sub(hipStream_t s, int64_t n, const double* X, int64_t ldx, const double* Y, int64_t ldy,
                double* Z, int64_t ldz);

// Block Gauss-Jordan on W = [G | R] (n x (n + nrhs), column-major, ldw);
// scratch is gj_scratch_bytes(n, n + nrhs) bytes of device memory.  With pre,
// the elimination first forms one right-hand-side column from the bordered
// Gram products, exactly as launch_border_combine with G1 = W and G2 = W + n ldw
// (the one-launch form does it in its first kernel).
struct GjCombine {
  double* g;         // A1^T b1 in, A^T J b out (n)
  const double* g2;  // A2^T b2 (n)
  double* gcol;      // the column of W that receives A^T J b
};
// Extra work of the one-launch form (n <= 2048 with right-hand sides,
// gj_one_launch): the loop state cleared first (and ||reset_xr||^2 into its
// scal[1] when reset_xr is given), as launch_state_reset, and columns
// [bcol0, bcol0 + nbt) of the result written row-major as well:
// bt[(c - bcol0) + r ldbt] = W[r, c].
struct GjExtras {
  LoopState* reset;
  const double* reset_xr;
  double* bt;
  int64_t ldbt, bcol0, nbt;
};
size_t gj_scratch_bytes(int64_t n, int64_t ncols);
bool gj_one_launch(int64_t n, int64_t nrhs);
void launch_gj(hipStream_t s, int64_t n, int64_t nrhs, double* W, int64_t ldw, void* scratch, int* bits,
               const GjCombine* pre = nullptr, const GjExtras* ex = nullptr);

// SP outer step kernels (k_sp.hip).
struct SpStepArgs {
  int64_t n;
  const double* Mrow;   // n x n row-major iteration matrix (paper form) or P (correction form)
  int64_t ldm;
  const double* c;      // n, paper form constant
  const double* H;      // n x n column-major A^T J A (RR metric, paper form), or null
  int64_t ldh;
  const double* g;      // A^T J b
  const double* x_ref;  // XREF metric
  double* xbuf0;
  double* xbuf1;
  double* x_out;        // the caller's x, written when the loop finishes
  const double* x0;     // paper form: the caller's x0 (null: zero), read by step 0
  const double* r;      // correction form: residual at x_k (n)
  double* partials;     // per-block metric partials, two sets of sp_step_blocks(n)
  int* nonfinite_part;  // per-block flags, two sets
  double* next_partials;// XREF: per-block partials of x_{k+1}'s metric (two sets), or null
  LoopState* st;
  int stop_rule;
  double tol;
  int64_t max_outer;
  int form;
  // mapped pinned host memory (device address) that the deciding launch also
  // writes done, status, iters and metric to, or null
  LoopState* mirror = nullptr;
};
int sp_step_blocks(int64_t n);
void launch_sp_step(hipStream_t s, const SpStepArgs& a, int64_t k);


// C = alpha X^T S Y + beta C0 (k_gemm.hip); S = diag(+1 for k < kneg, -1 after).
struct GemmTnArgs {
  int64_t M, N, K;
  const double* X;
  int64_t ldx;          // K x M, column-major
  const double* Y;
  int64_t ldy;          // K x N, column-major
  int64_t kneg;         // first negated row of Y (>= K: none)
  double alpha, beta;
  const double* C0;     // read iff beta != 0
  int64_t ldc0;
  double* C;
  int64_t ldc;
  const int* active;    // optional column mask
  const double* keep;   // inactive columns: C[:, j] = keep[:, j] (null: left as is)
  int64_t ldkeep;
};
void launch_gemm_tn(hipStream_t s, const GemmTnArgs& g);
// The same product on the persistent Gram kernel's plan (per-XCD row ranges,
// partial tiles reduced with the epilogue; k_gram.hip); false (nothing
// queued) when it does not apply (alignment, plan, or partials smaller than
// gemm_tn_pers_partials(K, M, N) doubles).
size_t gemm_tn_pers_partials(int64_t K, int64_t M, int64_t N);
bool launch_gemm_tn_pers(hipStream_t s, const GemmTnArgs& g, double* partials, size_t partial_doubles);

// Multi-right-hand-side helpers (k_multi.hip).
void launch_mat_copy(hipStream_t s, int64_t rows, int64_t cols, const double* X, int64_t ldx,
                     double* Y, int64_t ldy);
void launch_colnorm2(hipStream_t s, int64_t rows, int64_t cols, const double* V, int64_t ldv,
                     double* out);
void launch_fill_int(hipStream_t s, int64_t n, int value, int* dst);
struct MultiMetricArgs {
  int64_t n, N;
  const double* V;      // X_k (XREF) or R = H X_k - G (RR), n x N
  int64_t ldv;
  const double* Xref;   // XREF: n x N
  int64_t ldr;
  const double* den2;   // per column: ||x_ref_j||^2 (XREF) or ||g_j||^2 (RR)
  int stop_rule;
  double tol;
  int report;           // 1: only write metric[j] for every column
  int* active;
  int64_t* iters;
  double* metric;
  int* nactive;
  int* bits;
};
void launch_multi_metric(hipStream_t s, const MultiMetricArgs& a, int64_t k);

}  // namespace ils
