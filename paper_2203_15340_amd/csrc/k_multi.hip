// k_multi.hip -- per-column helpers of the multi-right-hand-side SP solve:
// matrix copies, column norms and the per-column stop test of Sec. 5 (RR,
// or the relative error to a reference), which retires converged columns.
#include "ils_common.hpp"

namespace ils {

__global__ __launch_bounds__(256) void k_mat_copy(int64_t rows, int64_t cols, const double* __restrict__ X,
                                                  int64_t ldx, double* __restrict__ Y, int64_t ldy) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t j = e / rows, i = e - j * rows;
    Y[i + j * ldy] = X ? X[i + j * ldx] : 0.0;
  }
}

void launch_mat_copy(hipStream_t s, int64_t rows, int64_t cols, const double* X, int64_t ldx, double* Y,
                     int64_t ldy) {
  if (rows <= 0 || cols <= 0) return;
  int64_t blocks = (rows * cols + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_mat_copy, dim3((unsigned)blocks), dim3(256), 0, s, rows, cols, X, ldx, Y, ldy);
}

__global__ void k_fill_int(int64_t n, int value, int* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = value;
}

void launch_fill_int(hipStream_t s, int64_t n, int value, int* dst) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)blocks), dim3(256), 0, s, n, value, dst);
}

// One workgroup per column.
__global__ __launch_bounds__(256) void k_colnorm2(int64_t rows, const double* __restrict__ V, int64_t ldv,
                                                  double* __restrict__ out) {
  __shared__ double red[4];
  const double* v = V + (int64_t)blockIdx.x * ldv;
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) a += v[i] * v[i];
  a = block_sum<256>(a, red);
  if (threadIdx.x == 0) out[blockIdx.x] = a;
}

void launch_colnorm2(hipStream_t s, int64_t rows, int64_t cols, const double* V, int64_t ldv, double* out) {
  if (cols <= 0) return;
  hipLaunchKernelGGL(k_colnorm2, dim3((unsigned)cols), dim3(256), 0, s, rows, V, ldv, out);
}

// One workgroup per column: the metric at x_k of column j (Sec. 5: RR =
// ||A^T J (b - A x_k)||^2 / ||A^T J b||^2, or ||x_k - x_ref|| / ||x_ref||).
// A column below tol is retired at outer count k; live columns are counted.
__global__ __launch_bounds__(256) void k_multi_metric(MultiMetricArgs a, int64_t k) {
  __shared__ double red[4];
  const int64_t j = blockIdx.x;
  if (!a.report && !a.active[j]) return;
  const double* v = a.V + j * a.ldv;
  const double* r = a.Xref ? a.Xref + j * a.ldr : nullptr;
  double s = 0.0;
  if (a.stop_rule == ILS_STOP_XREF) {
    for (int64_t i = threadIdx.x; i < a.n; i += 256) {
      const double d = v[i] - r[i];
      s += d * d;
    }
  } else {
    for (int64_t i = threadIdx.x; i < a.n; i += 256) s += v[i] * v[i];
  }
  s = block_sum<256>(s, red);
  if (threadIdx.x != 0) return;
  const double m = a.stop_rule == ILS_STOP_XREF ? sqrt(s) / sqrt(a.den2[j]) : s / a.den2[j];
  a.metric[j] = m;
  if (a.report) return;
  if (!isfinite(m)) {
    atomicOr(a.bits, kBitNonfinite);
    a.active[j] = 0;
    a.iters[j] = k;
  } else if (m < a.tol) {
    a.active[j] = 0;
    a.iters[j] = k;
  } else {
    atomicAdd(a.nactive, 1);
  }
}

void launch_multi_metric(hipStream_t s, const MultiMetricArgs& a, int64_t k) {
  if (a.N <= 0) return;
  hipLaunchKernelGGL(k_multi_metric, dim3((unsigned)a.N), dim3(256), 0, s, a, k);
}

}  // namespace ils
