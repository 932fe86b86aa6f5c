// ils_batched_api.hip -- host side of ils_sp_solve_batched: checks, the
// problem queue in device memory, and the persistent launch captured once in
// a hipGraph and replayed.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "ils_common.hpp"
#include "ils_runtime.hpp"
#include "k_batched.hpp"

using namespace ils;

#define HIPCHK(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return ILS_ERR_HIP; \
  } while (0)

namespace {

struct GraphKey {
  int64_t batch;
  int workgroups, stage_rows, precision, form, stop_rule;
  double tol;
  int64_t max_outer, slot_doubles, ldw, nmax;
  const void *probs, *order, *res, *work, *queue;
};

int ensure_pinned(ils_handle* h, size_t bytes) {
  if (h->pinned_cap >= bytes) return ILS_OK;
  if (h->pinned) (void)hipHostFree(h->pinned);
  h->pinned = nullptr;
  h->pinned_cap = 0;
  if (hipHostMalloc(&h->pinned, bytes, hipHostMallocDefault) != hipSuccess) return ILS_ERR_ALLOC;
  h->pinned_cap = bytes;
  return ILS_OK;
}

}  // namespace

namespace ils {
// The batched solve with the launch choices of `force` (tuning) or of the
// process-wide table.
int batched_solve(ils_handle* h, int64_t batch, const ils_problem* probs, const ils_opts* o, ils_info* infos,
                  const BatchCfg* force);
}  // namespace ils

extern "C" int ils_sp_solve_batched(ils_handle* h, int64_t batch, const ils_problem* probs,
                                    const ils_opts* o, ils_info* infos) {
  return batched_solve(h, batch, probs, o, infos, nullptr);
}

int ils::batched_solve(ils_handle* h, int64_t batch, const ils_problem* probs, const ils_opts* o, ils_info* infos,
                       const BatchCfg* force) {
  if (!h || batch < 1 || batch > (1 << 30) || !probs || !o || !infos) return ILS_ERR_ARG;
  // per-problem checks with the single-problem rules
  int64_t nmax = 1;
  for (int64_t i = 0; i < batch; ++i) {
    const ils_problem& P = probs[i];
    ils_opts oi = *o;
    oi.x_ref = P.x_ref;
    int st = check_problem(P.p, P.q, P.n, P.A, P.lda, P.b, P.x, &oi);
    if (st == ILS_OK && (P.n > kBatchMaxN || P.p + P.q > kBatchMaxM)) st = ILS_ERR_ARG;
    if (st != ILS_OK) {
      for (int64_t k = 0; k < batch; ++k) {
        memset(&infos[k], 0, sizeof(ils_info));
        infos[k].status = ILS_ERR_ARG;
        infos[k].rr = NAN;
        infos[k].rel_err = -1.0;
      }
      return ILS_ERR_ARG;
    }
    nmax = std::max(nmax, P.n);
  }
  HIPCHK(hipSetDevice(h->device));
  hipStream_t s = h->stream;
  int cus = 0;
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
  const BatchCfg bc = force ? *force : batched_cfg(o->precision, o->form, nmax, batch);
  const int workgroups = (int)std::min<int64_t>(batch, (int64_t)bc.wpc * cus);
  const int64_t ldw = nmax;
  const int64_t w_doubles = ldw * (2 * nmax + 1);
  const int64_t slot_doubles = (w_doubles + 4 * nmax + 31) / 32 * 32;

  BatchProblem* dprobs;
  int* dorder;
  BatchResult* dres;
  double* dwork;
  unsigned* dqueue;
  const bool fresh_queue = h->bufs[kBufBQueue].p == nullptr;
  int st;
  if ((st = h->need(kBufBProbs, sizeof(BatchProblem) * batch, (void**)&dprobs)) ||
      (st = h->need(kBufBOrder, sizeof(int) * batch, (void**)&dorder)) ||
      (st = h->need(kBufBRes, sizeof(BatchResult) * batch, (void**)&dres)) ||
      (st = h->need(kBufBWork, sizeof(double) * slot_doubles * workgroups, (void**)&dwork)) ||
      (st = h->need(kBufBQueue, 2 * sizeof(unsigned), (void**)&dqueue)))
    return st;
  if (fresh_queue) {
    HIPCHK(hipMemsetAsync(dqueue, 0, 2 * sizeof(unsigned), s));
  }

  // descriptors and the largest-first order, uploaded only when they change
  const size_t desc_bytes = sizeof(BatchProblem) * batch, order_bytes = sizeof(int) * batch;
  const size_t up_bytes = desc_bytes + order_bytes;
  if (h->batch_uploaded.size() != sizeof(ils_problem) * batch ||
      memcmp(h->batch_uploaded.data(), probs, sizeof(ils_problem) * batch) != 0 ||
      h->bkey.empty() || h->batch_order != bc.order) {
    if ((st = ensure_pinned(h, up_bytes))) return st;
    HIPCHK(hipStreamSynchronize(s));  // the staging area may still feed an earlier copy
    BatchProblem* hp = (BatchProblem*)h->pinned;
    for (int64_t i = 0; i < batch; ++i) {
      hp[i].p = probs[i].p;
      hp[i].q = probs[i].q;
      hp[i].n = probs[i].n;
      hp[i].lda = probs[i].lda;
      hp[i].A = probs[i].A;
      hp[i].b = probs[i].b;
      hp[i].x0 = probs[i].x0;
      hp[i].x_ref = probs[i].x_ref;
      hp[i].x = probs[i].x;
    }
    std::vector<int> order(batch);
    std::iota(order.begin(), order.end(), 0);
    if (bc.order == kBatchOrderLargest)
      std::stable_sort(order.begin(), order.end(),
                       [&](int x, int y) { return probs[x].n * probs[x].n * (probs[x].p + probs[x].n) >
                                                  probs[y].n * probs[y].n * (probs[y].p + probs[y].n); });
    h->batch_order = bc.order;
    memcpy((char*)h->pinned + desc_bytes, order.data(), order_bytes);
    HIPCHK(hipMemcpyAsync(dprobs, hp, desc_bytes, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dorder, (char*)h->pinned + desc_bytes, order_bytes, hipMemcpyHostToDevice, s));
    h->batch_uploaded.assign((const char*)probs, (const char*)probs + sizeof(ils_problem) * batch);
  }

  BatchArgs a;
  a.probs = dprobs;
  a.order = dorder;
  a.count = (int)batch;
  a.res = dres;
  a.work = dwork;
  a.slot_doubles = slot_doubles;
  a.w_doubles = w_doubles;
  a.ldw = ldw;
  a.nmax = nmax;
  a.queue = dqueue;
  a.precision = o->precision;
  a.form = o->form;
  a.stop_rule = o->stop_rule;
  a.tol = o->tol;
  a.max_outer = o->max_outer;

  GraphKey key;
  memset(&key, 0, sizeof(key));
  key.batch = batch;
  key.workgroups = workgroups;
  key.stage_rows = bc.stage_rows;
  key.precision = o->precision;
  key.form = o->form;
  key.stop_rule = o->stop_rule;
  key.tol = o->tol;
  key.max_outer = o->max_outer;
  key.slot_doubles = slot_doubles;
  key.ldw = ldw;
  key.nmax = nmax;
  key.probs = dprobs;
  key.order = dorder;
  key.res = dres;
  key.work = dwork;
  key.queue = dqueue;
  const bool same = h->bexec && h->bkey.size() == sizeof(key) && memcmp(h->bkey.data(), &key, sizeof(key)) == 0;
  if (!same) {
    if (h->bexec) (void)hipGraphExecDestroy(h->bexec);
    if (h->bgraph) (void)hipGraphDestroy(h->bgraph);
    h->bexec = nullptr;
    h->bgraph = nullptr;
    h->bkey.clear();
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    launch_batched(s, a, workgroups, bc.stage_rows);
    HIPCHK(hipStreamEndCapture(s, &h->bgraph));
    HIPCHK(hipGraphInstantiate(&h->bexec, h->bgraph, nullptr, nullptr, 0));
    h->bkey.assign((const char*)&key, (const char*)&key + sizeof(key));
  }
  HIPCHK(hipEventRecord(h->ev0, s));
  HIPCHK(hipGraphLaunch(h->bexec, s));
  HIPCHK(hipEventRecord(h->ev1, s));
  std::vector<BatchResult> res(batch);
  HIPCHK(hipMemcpyAsync(res.data(), dres, sizeof(BatchResult) * batch, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
  int first = ILS_OK;
  for (int64_t i = 0; i < batch; ++i) {
    ils_info& inf = infos[i];
    memset(&inf, 0, sizeof(inf));
    inf.status = res[i].status;
    inf.outer_iters = res[i].iters;
    inf.rr = (o->stop_rule == ILS_STOP_RR) ? res[i].metric : NAN;
    inf.rel_err = (o->stop_rule == ILS_STOP_XREF) ? res[i].metric : -1.0;
    inf.device_ms = ms;
    if (first == ILS_OK && res[i].status != ILS_OK) first = res[i].status;
  }
  return first;
}
