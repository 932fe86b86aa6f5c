// ils_runtime.hpp -- the handle behind the opaque ils_handle of include/ils.h
// and helpers shared by the solver drivers.
#pragma once
#include <vector>

#include "ils_common.hpp"

namespace ils {

// Workspace slots owned by a handle.
enum BufSlot {
  kBufG = 0,    // A^T J b
  kBufCn,       // squared column norms of A1
  kBufW,        // Gauss-Jordan work matrix / A1^T A1
  kBufM,        // iteration matrix, row-major
  kBufH,        // A^T J A (RR test in the paper form)
  kBufG2,       // A2^T A2
  kBufPart,     // Gram split-K partial tiles
  kBufX0,
  kBufX1,
  kBufT,        // m-vector scratch
  kBufR,        // n-vector scratch (residual / right-hand side)
  kBufSPart,    // per-block partial sums
  kBufSBad,     // per-block flags
  kBufW1,       // randomized inner state (w)
  kBufS1,       // randomized inner state (s)
  kBufZ,        // randomized inner state (z / beta)
  kBufIdx,      // pre-drawn index streams
  kBufMask,     // pre-drawn SCD subsets
  kBufPrefix,   // sampler prefix sums
  kBufA1f,      // FP32 copy of A1
  kBufDinv,     // inverted Gauss-Jordan pivot blocks
  kBufBProbs,   // batched: problem descriptors
  kBufBOrder,   // batched: processing order
  kBufBRes,     // batched: per-problem results
  kBufBWork,    // batched: per-workgroup slots
  kBufBQueue,   // batched: work-queue counters
  kBufMG,       // multi-RHS: A^T J B
  kBufMX0,      // multi-RHS: iterates (ping)
  kBufMX1,      // multi-RHS: iterates (pong)
  kBufMR,       // multi-RHS: residuals for the RR test
  kBufMAct,     // multi-RHS: active-column mask
  kBufMIters,   // multi-RHS: per-column outer counts
  kBufMMetric,  // multi-RHS: per-column stop metric
  kBufMDen,     // multi-RHS: per-column metric denominators
  kBufMBt,      // multi-RHS: B^T
  kBufA1f32,    // FP32 copy of A1 (mixed-precision RK-RGS inner sweeps)
  kBufRkb,      // blocked RK-RGS inner steps: slice partials, C, coefficients
  kBufRmW,      // multi-RHS RK-RGS: w of every right-hand side (p x nrhs)
  kBufRmS,      // multi-RHS RK-RGS: s (p x nrhs)
  kBufRmZ,      // multi-RHS RK-RGS: z (n x nrhs)
  kBufRmT,      // multi-RHS RK-RGS: inner targets (n x nrhs)
  kBufRmV,      // multi-RHS RK-RGS: w - s of a group (p x kMR), then A1^T of it (n x kMR)
  kBufRmF,      // multi-RHS RK-RGS: frozen flags, target norms
  kBufMC,       // prepared-A SP: P A^T J B
  kBufCount
};

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

}  // namespace ils

struct ils_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  ils::Buf bufs[ils::kBufCount];
  ils::LoopState* st = nullptr;       // device
  ils::LoopState* st_host = nullptr;  // pinned host mirror
  // mapped pinned host memory the SP step's deciding launch writes its
  // outcome to (host address, device address), so the SP solve reads it
  // without a device-to-host copy
  ils::LoopState* st_map = nullptr;
  ils::LoopState* st_map_dev = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  static constexpr int kPhases = 7;
  int profile = ILS_PROFILE_OFF;  // ILS_PROFILE_*
  hipEvent_t pev[kPhases + 1] = {};
  // SP outer launches queued before the first look at the loop state: the
  // previous solve's count plus the deciding launch (a guess; too few costs a
  // host round trip, too many a few launches that return at once)
  int64_t sp_queue = 8;
  // batched solver: pinned staging, last uploaded descriptors, captured launch
  void* pinned = nullptr;
  size_t pinned_cap = 0;
  std::vector<char> batch_uploaded;
  int batch_order = -1;  // processing-order policy of the uploaded order array
  hipGraph_t bgraph = nullptr;
  hipGraphExec_t bexec = nullptr;
  std::vector<char> bkey;
  void mark(int i) {
    if (profile == ILS_PROFILE_PHASES || (profile == ILS_PROFILE_GRAM && i == 1))
      (void)hipEventRecord(pev[i], stream);
  }
  // the event that closes the main Gram kernel (recorded between it and its
  // split-K reduction), or null when not profiling
  hipEvent_t gram_end_event() const { return profile != ILS_PROFILE_OFF ? pev[2] : nullptr; }
  // ils_info::device_ms of the single-problem solvers is measured only while
  // phase timing is on: an event record costs host time at the start of a
  // solve, while the device waits for its first kernel
  bool timing() const { return profile != ILS_PROFILE_OFF; }
  ~ils_handle();
  int need(int slot, size_t bytes, void** out);
};

struct ils_csr;

namespace ils {
// The matrix A = [A1; A2] as the solver drivers see it: dense column-major
// (A, lda) or sparse (sp: CSR plus the library's CSC copy).
struct MatOp {
  int64_t p = 0, q = 0, n = 0;
  const double* A = nullptr;
  int64_t lda = 0;
  const ils_csr* sp = nullptr;
};
int check_op(const MatOp& M, const double* b, const double* x, const ils_opts* o);
size_t mat_gram_partials(const MatOp& M);  // doubles of split-K scratch for mat_gram
void mat_colpass(hipStream_t s, const MatOp& M, const double* b, double* g, double* cn, int* bits);
// chk: the SP step's stopping test to repeat first (dense one-pass path), or null
void mat_residual(hipStream_t s, const MatOp& M, const double* b, const double* x, double* t, double* r,
                  const int* done, const SpStopCheck* chk = nullptr);
// G = A1^T A1 (second == 0) or A2^T A2 (second == 1).
void mat_gram(hipStream_t s, const MatOp& M, int second, int precision, void* part, double* G, int64_t ldg,
              hipEvent_t mid = nullptr);
void mat_rk_inner(hipStream_t st, const MatOp& M, const double* tgt, const double* cn, const int* j1,
                  const int* j2, int64_t count, double* w, double* s, double* z, const int* inner_done,
                  const int* outer_done);
void mat_rk_check(hipStream_t st, const MatOp& M, const double* w, const double* s, double* v, const double* tgt,
                  double* res2, double itol2, const double* tn2, int* inner_done, unsigned* arrive,
                  const int* skip);
int sp_solve_op(ils_handle* h, const MatOp& M, const double* b, const double* x0, double* x, const ils_opts* o,
                ils_info* info);
int rk_solve_op(ils_handle* h, const MatOp& M, const double* b, const double* x0, double* x, const ils_opts* o,
                ils_info* info);
int rgs_solve_op(ils_handle* h, const MatOp& M, const double* b, const double* x0, double* x, const ils_opts* o,
                 ils_info* info);

int check_problem(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda, const double* b,
                  const double* x, const ils_opts* o);
int finish_info(ils_handle* h, int64_t n, double* x, const ils_opts* o, int status, int64_t outer,
                int64_t inner, double metric, ils_info* info);
int setup_status(const LoopState& s);
int read_state(ils_handle* h);
}  // namespace ils
