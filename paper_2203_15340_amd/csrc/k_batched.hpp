// k_batched.hpp -- device-side descriptors and launcher of the batched solver.
#pragma once
#include "ils_common.hpp"

namespace ils {

constexpr int64_t kBatchMaxN = 256;   // largest n per problem in a batch
constexpr int64_t kBatchMaxM = 4096;  // largest p + q per problem (LDS residual vector)

// Mirror of ils_problem (include/ils.h), copied to the device.
struct BatchProblem {
  int64_t p, q, n, lda;
  const double* A;
  const double* b;
  const double* x0;
  const double* x_ref;
  double* x;
};

struct BatchResult {
  int status;
  int pad;
  int64_t iters;
  double metric;
};

struct BatchArgs {
  const BatchProblem* probs;
  const int* order;       // processing order (largest n first)
  int count;
  BatchResult* res;
  double* work;           // one slot per workgroup
  int64_t slot_doubles;
  int64_t w_doubles;      // W part of a slot: ldw x (2 nmax + 1)
  int64_t ldw;
  int64_t nmax;
  unsigned* queue;        // [0] next problem, [1] workgroups finished
  int precision;
  int form;
  int stop_rule;
  double tol;
  int64_t max_outer;
};

// stage_rows: rows of A per LDS stage of the Gram products (16, 32 or 64).
void launch_batched(hipStream_t s, const BatchArgs& a, int workgroups, int stage_rows);

// Launch choices of the batched solver, per (precision, form, n bucket,
// batch-size bucket): Gram stage rows, resident workgroups per CU (1 or 2)
// and the order problems are taken in (largest first, or as given).
enum { kBatchOrderLargest = 0, kBatchOrderGiven = 1 };
struct BatchCfg {
  int stage_rows = 32;
  int wpc = 2;
  int order = kBatchOrderLargest;
};
BatchCfg batched_cfg(int precision, int form, int64_t nmax, int64_t batch);

}  // namespace ils
