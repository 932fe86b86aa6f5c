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

void launch_batched(hipStream_t s, const BatchArgs& a, int workgroups);

}  // namespace ils
