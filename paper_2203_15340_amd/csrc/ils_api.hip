// ils_api.hip -- host runtime behind include/ils.h: handle, workspace,
// argument checks and the drivers that queue the gfx950 kernels.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>

#include "ils_common.hpp"
#include "ils_runtime.hpp"

using namespace ils;

// ------------------------------------------------------------------ handle
ils_handle::~ils_handle() {
  for (auto& b : bufs) if (b.p) (void)hipFree(b.p);
  if (st) (void)hipFree(st);
  if (st_host) (void)hipHostFree(st_host);
  if (st_map) (void)hipHostFree(st_map);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  for (auto& e : pev)
    if (e) (void)hipEventDestroy(e);
  if (bexec) (void)hipGraphExecDestroy(bexec);
  if (bgraph) (void)hipGraphDestroy(bgraph);
  if (pinned) (void)hipHostFree(pinned);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

int ils_handle::need(int slot, size_t bytes, void** out) {
  Buf& b = bufs[slot];
  if (b.cap < bytes) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    size_t want = bytes < 256 ? 256 : bytes;
    if (hipMalloc(&b.p, want) != hipSuccess) {
      b.p = nullptr;
      return ILS_ERR_ALLOC;
    }
    b.cap = want;
  }
  *out = b.p;
  return ILS_OK;
}

// ------------------------------------------------------------------ fixed scratch
// Workspace of the allocation-free entry point (ils_residual_noalloc): a
// file-scope device array, one copy on every device the library is loaded on,
// held until the process ends.  In host code `scratch` only names the array;
// its device address is looked up once per device (with that device current)
// by ils_create and kept in g_scratch_dev, and only that address is handed to
// kernels.
constexpr size_t kScratchDoubles = (size_t)1 << 20;  // 8 MiB
constexpr int kScratchDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];
static double* g_scratch_dev[kScratchDevices];
static std::mutex g_scratch_mu;

// Called with `device` current.
static int bind_scratch(int device) {
  if (device >= kScratchDevices) return ILS_OK;  // no fixed scratch there: the no-alloc call rejects it
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return ILS_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ILS_ERR_HIP;
  g_scratch_dev[device] = (double*)p;
  return ILS_OK;
}

static double* scratch_of(int device) {
  if (device < 0 || device >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_dev[device];
}

extern "C" int ils_create(ils_handle** out, int device_ordinal, void* hip_stream) {
  if (!out) return ILS_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device_ordinal < 0 || device_ordinal >= ndev)
    return ILS_ERR_ARG;
  if (hipSetDevice(device_ordinal) != hipSuccess) return ILS_ERR_HIP;
  if (bind_scratch(device_ordinal) != ILS_OK) return ILS_ERR_HIP;
  ils_handle* h = new ils_handle();
  h->device = device_ordinal;
  if (hip_stream) {
    h->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      delete h;
      return ILS_ERR_HIP;
    }
    h->own_stream = true;
  }
  if (hipMalloc((void**)&h->st, sizeof(LoopState)) != hipSuccess ||
      hipHostMalloc((void**)&h->st_host, sizeof(LoopState), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&h->st_map, sizeof(LoopState), hipHostMallocMapped | hipHostMallocCoherent) !=
          hipSuccess ||
      hipHostGetDevicePointer((void**)&h->st_map_dev, h->st_map, 0) != hipSuccess ||
      hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) {
    delete h;
    return ILS_ERR_ALLOC;
  }
  for (auto& e : h->pev) {
    if (hipEventCreate(&e) != hipSuccess) {
      delete h;
      return ILS_ERR_ALLOC;
    }
  }
  *out = h;
  return ILS_OK;
}

extern "C" int ils_destroy(ils_handle* h) {
  if (!h) return ILS_ERR_ARG;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return ILS_OK;
}

extern "C" void ils_opts_default(ils_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->tol = 1e-6;
  o->stop_rule = ILS_STOP_RR;
  o->form = ILS_FORM_PAPER;
  o->precision = ILS_PREC_FP64;
  o->sampling = ILS_SAMPLE_UNIFORM;
  o->x_ref = nullptr;
  o->max_outer = 20000;
  o->max_inner = -1;
  o->inner_tol = -1.0;
  o->inner_check = -1;
  o->seed = 0;
  o->stream_offset = 0;
  o->alpha = 0;
}

extern "C" const char* ils_status_string(int status) {
  switch (status) {
    case ILS_OK: return "ok";
    case ILS_ERR_ARG: return "invalid argument";
    case ILS_ERR_NOT_SPD: return "A1^T A1 (hence A^T J A) is not positive definite";
    case ILS_ERR_NO_CONVERGENCE: return "outer iteration limit reached";
    case ILS_ERR_NONFINITE: return "non-finite value in the input or an iterate";
    case ILS_ERR_HIP: return "HIP runtime error";
    case ILS_ERR_ALLOC: return "device allocation failed";
    default: return "unknown status";
  }
}

// ------------------------------------------------------------------ shared checks
int ils::check_problem(int64_t p, int64_t q, int64_t n, const double* A, int64_t lda, const double* b,
                       const double* x, const ils_opts* o) {
  if (!A || !b || !x || !o) return ILS_ERR_ARG;
  if (n < 1 || q < 0 || p < n || lda < p + q) return ILS_ERR_ARG;
  if (n > (int64_t)1 << 20 || p + q > ((int64_t)1 << 40)) return ILS_ERR_ARG;
  if (o->stop_rule < ILS_STOP_RR || o->stop_rule > ILS_STOP_FIXED) return ILS_ERR_ARG;
  if (o->stop_rule != ILS_STOP_FIXED && !(o->tol > 0.0)) return ILS_ERR_ARG;
  if (o->stop_rule == ILS_STOP_XREF && !o->x_ref) return ILS_ERR_ARG;
  if (o->max_outer < 0) return ILS_ERR_ARG;
  if (o->form != ILS_FORM_PAPER && o->form != ILS_FORM_CORRECTION) return ILS_ERR_ARG;
  if (o->precision != ILS_PREC_FP64 && o->precision != ILS_PREC_MIXED) return ILS_ERR_ARG;
  if (o->precision == ILS_PREC_MIXED && o->form != ILS_FORM_CORRECTION) return ILS_ERR_ARG;
  if (o->sampling != ILS_SAMPLE_UNIFORM && o->sampling != ILS_SAMPLE_NORM) return ILS_ERR_ARG;
  return ILS_OK;
}

static int fail(ils_info* info, int st) {
  if (info) {
    memset(info, 0, sizeof(*info));
    info->status = st;
    info->rr = NAN;
    info->rel_err = -1.0;
  }
  return st;
}

#define HIPCHK(expr)                           \
  do {                                         \
    if ((expr) != hipSuccess) return ILS_ERR_HIP; \
  } while (0)

// Relative error ||x - x_ref|| / ||x_ref|| on the device.
__global__ __launch_bounds__(1024) void k_relerr(int64_t n, const double* __restrict__ x,
                                                 const double* __restrict__ xr, double* out) {
  __shared__ double red0[16], red1[16];
  double a = 0.0, c = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double d = x[i] - xr[i];
    a += d * d;
    c += xr[i] * xr[i];
  }
  a = block_sum<1024>(a, red0);
  c = block_sum<1024>(c, red1);
  if (threadIdx.x == 0) out[0] = sqrt(a) / sqrt(c);
}

int ils::finish_info(ils_handle* h, int64_t n, double* x, const ils_opts* o, int status,
                     int64_t outer, int64_t inner, double metric, ils_info* info) {
  if (!info) return status;
  info->status = status;
  info->pad = 0;
  info->outer_iters = outer;
  info->inner_iters = inner;
  info->rr = (o->stop_rule == ILS_STOP_RR) ? metric : NAN;
  info->rel_err = -1.0;
  if (o->stop_rule == ILS_STOP_XREF && (status == ILS_OK || status == ILS_ERR_NO_CONVERGENCE)) {
    info->rel_err = metric;  // the stop quantity is the relative error of the returned iterate
  } else if (o->x_ref && status != ILS_ERR_ARG && status != ILS_ERR_NOT_SPD) {
    hipLaunchKernelGGL(k_relerr, dim3(1), dim3(1024), 0, h->stream, n, (const double*)x, o->x_ref,
                       &h->st->scal[7]);
    double v = -1.0;
    if (hipMemcpyAsync(&v, &h->st->scal[7], sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return ILS_ERR_HIP;
    info->rel_err = v;
  }
  float ms = 0.0f;
  info->device_ms = (h->timing() && hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) ? ms : 0.0;
  return status;
}

// Status of the setup kernels (non-finite input, pivot failure).
int ils::setup_status(const LoopState& s) {
  if (s.bits & kBitNonfinite) return ILS_ERR_NONFINITE;
  if (s.bits & kBitNotSpd) return ILS_ERR_NOT_SPD;
  if (s.bits & kBitStall) return ILS_ERR_HIP;
  return ILS_OK;
}

// Wait for the handle's stream: poll it for up to 20 ms, then block.  A
// blocking wait sleeps and is woken well after the work ends, time the
// device then spends idle before the caller's next solve reaches it.
static int stream_wait(hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  while (std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(20)) {
    const hipError_t e = hipStreamQuery(s);
    if (e == hipSuccess) return ILS_OK;
    if (e != hipErrorNotReady) return ILS_ERR_HIP;
  }
  return hipStreamSynchronize(s) == hipSuccess ? ILS_OK : ILS_ERR_HIP;
}

int ils::read_state(ils_handle* h) {
  HIPCHK(hipMemcpyAsync(h->st_host, h->st, sizeof(LoopState), hipMemcpyDeviceToHost, h->stream));
  return stream_wait(h->stream);
}

// ------------------------------------------------------------------ SP
int ils::sp_solve_op(ils_handle* h, const MatOp& M, const double* b, const double* x0, double* x,
                     const ils_opts* o, ils_info* info) {
  if (!h) return fail(info, ILS_ERR_ARG);
  int st = check_op(M, b, x, o);
  if (st != ILS_OK) return fail(info, st);
  if (hipSetDevice(h->device) != hipSuccess) return fail(info, ILS_ERR_HIP);
  hipStream_t s = h->stream;
  const int64_t p = M.p, q = M.q, n = M.n;
  const int64_t m = p + q;
  const bool paper = o->form == ILS_FORM_PAPER;
  const bool need_h = paper && o->stop_rule == ILS_STOP_RR;
  const int64_t ldw = n;
  const int64_t nrhs = paper ? n + 1 : n;
  const int nblk = sp_step_blocks(n);
  double *g, *W, *Mrow, *H = nullptr, *xb0, *xb1, *tv, *rv, *spart, *dinv;
  void* part;
  int* sbad;
  const size_t part_bytes = mat_gram_partials(M) * sizeof(double);
  if ((st = h->need(kBufG, sizeof(double) * n, (void**)&g)) ||
      (st = h->need(kBufW, sizeof(double) * ldw * (n + nrhs), (void**)&W)) ||
      (st = h->need(kBufM, sizeof(double) * n * n, (void**)&Mrow)) ||
      (need_h && (st = h->need(kBufH, sizeof(double) * n * n, (void**)&H))) ||
      (st = h->need(kBufPart, part_bytes, &part)) ||
      (st = h->need(kBufX0, sizeof(double) * n, (void**)&xb0)) ||
      (st = h->need(kBufX1, sizeof(double) * n, (void**)&xb1)) ||
      (st = h->need(kBufT, sizeof(double) * residual_scratch(m, n), (void**)&tv)) ||
      (st = h->need(kBufR, sizeof(double) * n, (void**)&rv)) ||
      (st = h->need(kBufSPart, sizeof(double) * 4 * nblk, (void**)&spart)) ||
      (st = h->need(kBufSBad, sizeof(int) * 2 * nblk, (void**)&sbad)) ||
      (st = h->need(kBufDinv, gj_scratch_bytes(n, n + nrhs), (void**)&dinv)))
    return fail(info, st);
  // mixed precision: scratch for the FP32 copy of A1 when the launch table's
  // mixed Gram entry reads one (dense A; the paper form is FP64 only)
  float* a1f = nullptr;
  if (!M.sp && !paper && o->precision == ILS_PREC_MIXED && gram_f32_uses_copy(n, p) &&
      (st = h->need(kBufA1f32, sizeof(float) * gram_f32_copy_ld(p) * n, (void**)&a1f)))
    return fail(info, st);

  if (h->timing()) HIPCHK(hipEventRecord(h->ev0, s));
  h->mark(0);
  LoopState* ds = h->st;
  // dense paper form: A^T J b = A1^T b1 - A2^T b2 comes from the Gram
  // products of the bordered blocks [A1 b1] and [A2 b2], so A is read once.
  // The Gram launch touches no loop state, so it goes first in every form:
  // the device starts on it while the host queues the rest of the solve.
  const bool bordered = paper && !M.sp;
  hipEvent_t mid = h->gram_end_event();
  const double* xr = o->stop_rule == ILS_STOP_XREF ? o->x_ref : nullptr;
  if (a1f) {
    // mixed precision through the FP32 copy: the column pass writes the copy
    // of A1 while it reads A, then the Gram kernel reads only the copy
    launch_state_reset(s, ds, n, xr);
    launch_colpass(s, p, q, n, M.A, M.lda, b, g, nullptr, &ds->bits, a1f, gram_f32_copy_ld(p));
    h->mark(1);
    launch_gram_f32_on_copy(s, p, n, a1f, (float*)part, W, ldw, mid);
    if (o->stop_rule == ILS_STOP_RR) launch_norm2(s, n, g, &ds->scal[0]);
  } else {
    h->mark(1);
    if (bordered)  // A1^T A1, A1^T b1 and A2^T A2, A2^T b2 in one launch pair
      launch_gram2_f64(s, n, M.lda, ldw, (double*)part, mid, p, M.A, b, W, g, q, M.A + p, b + p, W + n * ldw,
                       rv);
    else  // A1^T A1 for [A1^T A1 | A2^T A2 | A^T J b] or [A1^T A1 | I]
      mat_gram(s, M, 0, o->precision, part, W, ldw, mid);
    // the bordered form's one-launch elimination clears the loop state in its
    // first kernel (nothing before it reads or raises the state's bits)
    if (!(bordered && gj_one_launch(n, nrhs))) launch_state_reset(s, ds, n, xr);
    if (!bordered) {
      mat_colpass(s, M, b, g, nullptr, &ds->bits);
      if (o->stop_rule == ILS_STOP_RR) launch_norm2(s, n, g, &ds->scal[0]);
    }
  }
  h->mark(3);
  GjCombine pre{g, rv, W + 2 * n * ldw};  // bordered: A^T J b formed by the elimination's first kernel
  if (bordered) {
    if (need_h) launch_sub(s, n, W, ldw, W + n * ldw, ldw, H, n);
  } else if (paper) {
    mat_gram(s, M, 1, ILS_PREC_FP64, part, W + n * ldw, ldw);
    launch_copy_cols(s, n, 1, g, n, W + 2 * n * ldw, ldw);
    if (need_h) launch_sub(s, n, W, ldw, W + n * ldw, ldw, H, n);
  } else {
    launch_eye(s, n, W + n * ldw, ldw);
  }
  h->mark(4);
  // the one-launch elimination also writes B (or P) row-major for the steps
  const bool one = gj_one_launch(n, nrhs);
  const GjExtras ex{bordered ? ds : nullptr, xr, Mrow, n, n, n};
  launch_gj(s, n, nrhs, W, ldw, dinv, &ds->bits, bordered ? &pre : nullptr, one ? &ex : nullptr);
  if (bordered && o->stop_rule == ILS_STOP_RR) launch_norm2(s, n, g, &ds->scal[0]);
  h->mark(5);
  if (!one) launch_transpose(s, n, n, W + n * ldw, ldw, Mrow, n);
  if (!paper) launch_fill_vec(s, n, x0, xb0);  // the paper form's step 0 reads x0 itself
  h->mark(6);

  SpStepArgs a;
  a.n = n;
  a.Mrow = Mrow;
  a.ldm = n;
  a.c = W + 2 * n * ldw;
  a.H = H;
  a.ldh = n;
  a.g = g;
  a.x_ref = o->x_ref;
  a.xbuf0 = xb0;
  a.xbuf1 = xb1;
  a.x_out = x;
  a.x0 = x0;
  a.r = rv;
  a.partials = spart;
  a.nonfinite_part = sbad;
  // correction form with a test that does not need r_{k+1}: x_{k+1}'s metric
  // partials as well, for the residual's skip test
  const bool test_next = !paper && o->stop_rule != ILS_STOP_RR;
  a.next_partials = (test_next && o->stop_rule == ILS_STOP_XREF) ? spart + 2 * nblk : nullptr;
  a.st = ds;
  a.stop_rule = o->stop_rule;
  a.tol = o->tol;
  a.max_outer = o->max_outer;
  a.form = o->form;
  a.mirror = h->st_map_dev;
  *(volatile int*)&h->st_map->done = 0;  // the previous solve's work has drained

  // launch k computes x_{k+1} and decides on x_{k-1}; launch max_outer + 1
  // only decides
  const int64_t nlaunch = o->max_outer + 2;
  int64_t k = 0, chunk = h->sp_queue;
  while (true) {
    const int64_t kend = std::min(k + chunk, nlaunch);
    for (; k < kend; ++k) {
      if (!paper && k == 0 && !x0) {
        // r_0 at x_0 = 0 is A^T J b, which the column pass formed
        SpStepArgs a0 = a;
        a0.r = g;
        launch_sp_step(s, a0, k);
        continue;
      }
      if (!paper && k <= o->max_outer) {
        // skipped on the device when the loop is going to end without r_k:
        // at x_{k-1} (launch k's test) or, for a test that does not need
        // r_k, at x_k (launch k + 1's test by the metric or the step limit)
        SpStopCheck chk{spart + ((k - 1) & 1) * nblk, sbad + ((k - 1) & 1) * nblk, nullptr, nblk, o->stop_rule,
                        o->tol, k - 1, o->max_outer, ds->scal, &ds->resid_skip};
        if (test_next) chk.part_next = a.next_partials ? a.next_partials + ((k - 1) & 1) * nblk : spart;
        mat_residual(s, M, b, k & 1 ? xb1 : xb0, tv, rv, &ds->done, k >= 1 ? &chk : nullptr);
      }
      launch_sp_step(s, a, k);
    }
    if (h->timing()) HIPCHK(hipEventRecord(h->ev1, s));
    // the deciding launch wrote its outcome to the mapped mirror: once the
    // stream has drained it is read there, with no copy; otherwise (a setup
    // kernel raised a bit, or more launches are needed) the state is copied
    if ((st = stream_wait(s))) return fail(info, st);
    if (*(volatile int*)&h->st_map->done) {
      h->st_host->done = h->st_map->done;
      h->st_host->status = h->st_map->status;
      h->st_host->iters = h->st_map->iters;
      h->st_host->metric = h->st_map->metric;
      h->st_host->bits = 0;
      break;
    }
    if ((st = read_state(h))) return fail(info, st);
    if (h->st_host->done || h->st_host->bits || k >= nlaunch) break;
    chunk = std::min<int64_t>(chunk * 2, 64);
  }
  h->mark(7);
  const LoopState& hs = *h->st_host;
  st = setup_status(hs);
  if (st != ILS_OK) return fail(info, st);
  if (!hs.done) return fail(info, ILS_ERR_HIP);  // every queued step ran without finishing
  st = hs.status;
  h->sp_queue = std::min<int64_t>(std::max<int64_t>(hs.iters + 2, 4), 64);
  return finish_info(h, n, x, o, st, hs.iters, 0, hs.metric, info);
}

extern "C" int ils_sp_solve(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                            const double* b, const double* x0, double* x, const ils_opts* o, ils_info* info) {
  MatOp M;
  M.p = p;
  M.q = q;
  M.n = n;
  M.A = A;
  M.lda = lda;
  return sp_solve_op(h, M, b, x0, x, o, info);
}

// ------------------------------------------------------------------ components
extern "C" int ils_gram(ils_handle* h, int64_t r0, int64_t r1, int64_t n, const double* A, int64_t lda,
                        double* G, int64_t ldg, int32_t precision) {
  if (!h || !A || !G || n < 1 || r0 < 0 || r1 < r0 || lda < r1 || ldg < n) return ILS_ERR_ARG;
  if (precision != ILS_PREC_FP64 && precision != ILS_PREC_MIXED) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  void* part;
  int st = h->need(kBufPart, gram_partials_size(n, r1 - r0) * sizeof(double), &part);
  if (st) return st;
  const int64_t K = r1 - r0;
  if (precision == ILS_PREC_MIXED && gram_f32_uses_copy(n, K)) {
    float* a1f;
    if ((st = h->need(kBufA1f32, sizeof(float) * gram_f32_copy_ld(K) * n, (void**)&a1f))) return st;
    launch_gram_f32_copy(h->stream, K, n, A + r0, lda, a1f, (float*)part, G, ldg);
  } else if (precision == ILS_PREC_MIXED) {
    launch_gram_f32(h->stream, K, n, A + r0, lda, (float*)part, G, ldg);
  } else {
    launch_gram_f64(h->stream, K, n, A + r0, lda, (double*)part, G, ldg);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return ILS_OK;
}

extern "C" int ils_colpass(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                           const double* b, double* g, double* colnorm2) {
  if (!h || !A || !b || !g || n < 1 || p < 0 || q < 0 || lda < p + q) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  HIPCHK(hipMemsetAsync(h->st, 0, sizeof(LoopState), h->stream));
  launch_colpass(h->stream, p, q, n, A, lda, b, g, colnorm2, &h->st->bits);
  int st = read_state(h);
  if (st) return st;
  return setup_status(*h->st_host);
}

extern "C" int ils_residual(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A, int64_t lda,
                            const double* b, const double* x, double* r) {
  if (!h || !A || !b || !x || !r || n < 1 || p < 0 || q < 0 || lda < p + q) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  double* tv;
  int st = h->need(kBufT, sizeof(double) * residual_scratch(p + q, n), (void**)&tv);
  if (st) return st;
  launch_residual(h->stream, p, q, n, A, lda, b, x, tv, r, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return ILS_OK;
}

extern "C" int ils_residual_noalloc(ils_handle* h, int64_t p, int64_t q, int64_t n, const double* A,
                                    int64_t lda, const double* b, const double* x, double* r) {
  if (!h || !A || !b || !x || !r || n < 1 || p < 0 || q < 0 || lda < p + q) return ILS_ERR_ARG;
  // the default launch choice (not the tuning table's), so the workspace
  // bound stated in ils.h holds
  if (residual_scratch_cfg(p + q, n, ResidCfg{}) > kScratchDoubles) return ILS_ERR_ARG;
  double* tv = scratch_of(h->device);
  if (!tv) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  launch_residual_cfg(h->stream, p, q, n, A, lda, b, x, tv, r, nullptr, ResidCfg{});
  HIPCHK(hipGetLastError());
  return ILS_OK;
}

extern "C" int ils_spd_solve(ils_handle* h, int64_t n, int64_t nrhs, const double* G, int64_t ldg,
                             const double* R, int64_t ldr, double* X, int64_t ldx) {
  if (!h || !G || !R || !X || n < 1 || nrhs < 1 || ldg < n || ldr < n || ldx < n) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  double *W, *dinv;
  int st;
  if ((st = h->need(kBufW, sizeof(double) * n * (n + nrhs), (void**)&W)) ||
      (st = h->need(kBufDinv, gj_scratch_bytes(n, n + nrhs), (void**)&dinv)))
    return st;
  HIPCHK(hipMemsetAsync(h->st, 0, sizeof(LoopState), h->stream));
  launch_copy_cols(h->stream, n, n, G, ldg, W, n);
  launch_copy_cols(h->stream, n, nrhs, R, ldr, W + n * n, n);
  launch_gj(h->stream, n, nrhs, W, n, dinv, &h->st->bits);
  launch_copy_cols(h->stream, n, nrhs, W + n * n, n, X, ldx);
  if ((st = read_state(h))) return st;
  return setup_status(*h->st_host);
}

// ------------------------------------------------------------------ instrumentation
extern "C" int ils_set_profiling(ils_handle* h, int mode) {
  if (!h || mode < ILS_PROFILE_OFF || mode > ILS_PROFILE_GRAM) return ILS_ERR_ARG;
  h->profile = mode;
  return ILS_OK;
}

extern "C" int ils_get_phase_times(ils_handle* h, double* ms, int count) {
  if (!h || !ms || count < 0) return ILS_ERR_ARG;
  if (h->profile == ILS_PROFILE_OFF) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  const bool all = h->profile == ILS_PROFILE_PHASES;
  HIPCHK(hipEventSynchronize(h->pev[all ? ils_handle::kPhases : 2]));
  const int nph = count < ils_handle::kPhases ? count : ils_handle::kPhases;
  for (int i = 0; i < nph; ++i) {
    float v = 0.0f;
    if (all || i == 1) HIPCHK(hipEventElapsedTime(&v, h->pev[i], h->pev[i + 1]));
    ms[i] = (all || i == 1) ? (double)v : NAN;
  }
  return nph;
}
