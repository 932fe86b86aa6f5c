// k_sp.hip -- one outer step of the SP iteration (Algorithm 1, step 6) with
// its stopping test, as a single launch that needs no host round trip.
//
// Launch k reads x_k and writes x_{k+1}:
//   paper form      x_{k+1} = B x_k + c            (B = (A1^T A1)^{-1} A2^T A2)
//   correction form x_{k+1} = x_k + P r_k          (P = (A1^T A1)^{-1},
//                                                    r_k = A^T J (b - A x_k))
// Each workgroup handles four rows (one per wave) and also writes its partial
// sum of the stop quantity at x_k (RR of Sec. 5, or the relative error
// against x_ref).  The stopping test for x_k is taken at the start of launch
// k + 1: every workgroup adds the partials of launch k in the same fixed
// order, so all reach the same decision without atomics or fences, and
// workgroup 0 records it in LoopState; the deciding launch also copies the
// returned iterate into the caller's x.  (The correction form's residual
// queued before launch k + 1 repeats the test that ends the loop: on x_{k+1}
// from the partials launch k also writes for it (relative error, fixed
// count), or on x_k (RR, which needs that residual), so the pass over A for
// an iterate the loop will not use is skipped.)  The host queues several steps ahead;
// a launch that finds the loop finished by an EARLIER launch returns at once.
// LoopState::done holds the deciding launch's index + 1, so a workgroup of the
// deciding launch itself that starts after workgroup 0's store is visible
// still takes the decision and writes its rows of x.
#include "ils_common.hpp"

namespace ils {

// kSpRows rows per workgroup, one wave each (2 and 8 measured slower at
// n = 1000: 70-74 us for the 7 steps of a solve against 65-68 us)

// Dot product of a contiguous row with v by one wave: each lane issues
// sixteen loads per round before using them (a 1000-long row is one round);
// lane partials are added by a fixed butterfly.
constexpr int kDotDepth = 16;

// The first round's loads alone, so a caller can issue them early, and the
// rest of dot_row from there (the same sums in the same order).
__device__ inline void dot_first(const double* row_, const double* v_, int64_t n, int lane,
                                 double (&rv)[kDotDepth], double (&vv)[kDotDepth]) {
  const auto row = glb(row_);
  const auto v = glb(v_);
#pragma unroll
  for (int u = 0; u < kDotDepth; ++u) {
    const int64_t j = lane + u * kWave;
    rv[u] = j < n ? row[j] : 0.0;
    vv[u] = (v_ && j < n) ? v[j] : 0.0;  // v_ null: the zero vector
  }
}
__device__ inline double dot_rest(const double* row_, const double* v_, int64_t n, int lane,
                                  const double (&rv0)[kDotDepth], const double (&vv0)[kDotDepth]) {
  const auto row = glb(row_);
  const auto v = glb(v_);
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kDotDepth; ++u) s = fma(rv0[u], vv0[u], s);
  for (int64_t j0 = kDotDepth * kWave; j0 < n; j0 += kDotDepth * kWave) {
    double rv[kDotDepth], vv[kDotDepth];
#pragma unroll
    for (int u = 0; u < kDotDepth; ++u) {
      const int64_t j = j0 + lane + u * kWave;
      rv[u] = j < n ? row[j] : 0.0;
      vv[u] = (v_ && j < n) ? v[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kDotDepth; ++u) s = fma(rv[u], vv[u], s);
  }
  return wave_sum(s);
}

__device__ inline double dot_row(const double* row_, const double* v_, int64_t n, int lane) {
  const auto row = glb(row_);
  const auto v = glb(v_);
  double s = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += kDotDepth * kWave) {
    double rv[kDotDepth], vv[kDotDepth];
#pragma unroll
    for (int u = 0; u < kDotDepth; ++u) {
      const int64_t j = j0 + lane + u * kWave;
      rv[u] = j < n ? row[j] : 0.0;
      vv[u] = j < n ? v[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kDotDepth; ++u) s = fma(rv[u], vv[u], s);
  }
  return wave_sum(s);
}

__global__ __launch_bounds__(kSpThreads) void k_sp_step(SpStepArgs a, int64_t k) {
  LoopState* st = a.st;
  const int decided = *(volatile int*)&st->done;  // 0, or deciding launch + 1
  if ((decided != 0 && (int64_t)decided <= k) || *(volatile int*)&st->bits) return;
  __shared__ double tred[kSpThreads / kWave];
  const unsigned nblk = gridDim.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * kSpRows + w;
  // paper form, step 0: x_0 is read from the caller's x0 (null: zero) and
  // copied to the first buffer here, so no separate fill launch is needed
  const bool first = k == 0 && a.form == ILS_FORM_PAPER;
  const double* xk = first ? a.x0 : ((k & 1) ? a.xbuf1 : a.xbuf0);
  const double* row = a.Mrow + i * a.ldm;
  const double* v = (a.form == ILS_FORM_PAPER) ? xk : a.r;
  // this step's row loads go out first; their latency overlaps the stopping
  // test of the previous step
  double rv0[kDotDepth], vv0[kDotDepth];
  // x_0 = 0 in the paper form: x_1 = c, the rows of B are not read
  const bool zero_v = first && !a.x0;
  if (i < a.n && !zero_v) dot_first(row, v, a.n, lane, rv0, vv0);
  if (k >= 1) {
    // stopping test for x_{k-1} from the partials of launch k - 1: strided
    // per thread, then the block tree (the same order in every workgroup)
    const int64_t kk = k - 1;
    const double* part = a.partials + (kk & 1) * nblk;
    const int* pbad = a.nonfinite_part + (kk & 1) * nblk;
    double tot = 0.0;
    int anybad = 0;
    for (unsigned bkt = threadIdx.x; bkt < nblk; bkt += kSpThreads) {
      tot += part[bkt];
      anybad |= pbad[bkt];
    }
    tot = block_sum<kSpThreads>(tot, tred);
    anybad = __syncthreads_or(anybad);
    const double metric = sp_metric(tot, a.stop_rule, st->scal);
    int done = 0, status = ILS_OK;
    int64_t iters = kk;
    if (a.stop_rule != ILS_STOP_FIXED && metric < a.tol) {
      done = 1;
    } else if (kk == a.max_outer) {
      done = 1;
      status = (a.stop_rule == ILS_STOP_FIXED) ? ILS_OK : ILS_ERR_NO_CONVERGENCE;
    } else if (anybad) {
      done = 1;
      status = ILS_ERR_NONFINITE;
      iters = kk + 1;
    }
    if (done) {
      // the returned iterate goes straight to the caller's x
      const double* xs = (iters & 1) ? a.xbuf1 : a.xbuf0;
      if ((threadIdx.x & 63) == 0 && i < a.n) a.x_out[i] = xs[i];
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int dv = (int)(k < INT_MAX - 1 ? k + 1 : INT_MAX);
        st->metric = metric;
        st->status = status;
        st->iters = iters;
        st->done = dv;
        if (a.mirror) {
          // the host reads these once the stream has drained
          a.mirror->metric = metric;
          a.mirror->status = status;
          a.mirror->iters = iters;
          __hip_atomic_store(&a.mirror->done, dv, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
      }
      return;
    }
  }
  double* xn = (k & 1) ? a.xbuf0 : a.xbuf1;
  double mp = 0.0, mpn = 0.0;
  int bad = 0;
  if (i < a.n) {
    const double dot = zero_v ? 0.0 : dot_rest(row, v, a.n, lane, rv0, vv0);
    const double xki = xk ? xk[i] : 0.0;
    if (first && lane == 0) a.xbuf0[i] = xki;
    const double xi = (a.form == ILS_FORM_PAPER) ? dot + a.c[i] : xki + dot;
    if (a.stop_rule == ILS_STOP_XREF) {
      const double d = xki - a.x_ref[i];
      mp = d * d;
    } else if (a.stop_rule == ILS_STOP_RR) {
      // (A^T J b - A^T J A x_k)_i in the paper form (A^T J A symmetric), r_k in
      // the correction form
      const double ri = (a.form == ILS_FORM_PAPER) ? a.g[i] - (xk ? dot_row(a.H + i * a.ldh, xk, a.n, lane) : 0.0)
                                                   : a.r[i];
      mp = ri * ri;
    }
    if (a.next_partials) {
      // x_{k+1}'s relative-error partial, the same value launch k + 1 forms
      const double dn = xi - a.x_ref[i];
      mpn = dn * dn;
    }
    if (lane == 0) xn[i] = xi;
    bad = !isfinite(xi);
  }
  __shared__ double red[kSpRows], redn[kSpRows];
  __shared__ int redb[kSpRows];
  if (lane == 0) {
    red[w] = mp;
    redn[w] = mpn;
    redb[w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = red[0], sumn = redn[0];
    int anyb = redb[0];
#pragma unroll
    for (int q = 1; q < kSpRows; ++q) {
      sum += red[q];
      sumn += redn[q];
      anyb |= redb[q];
    }
    a.partials[(k & 1) * nblk + blockIdx.x] = sum;
    a.nonfinite_part[(k & 1) * nblk + blockIdx.x] = anyb;
    if (a.next_partials) a.next_partials[(k & 1) * nblk + blockIdx.x] = sumn;
  }
}

int sp_step_blocks(int64_t n) { return (int)((n + kSpRows - 1) / kSpRows); }

void launch_sp_step(hipStream_t s, const SpStepArgs& a, int64_t k) {
  hipLaunchKernelGGL(k_sp_step, dim3((unsigned)sp_step_blocks(a.n)), dim3(kSpThreads), 0, s, a, k);
}

}  // namespace ils
