// k_batched.hip -- many small ILS problems in one persistent launch (gfx950).
//
// Each workgroup takes problems from an atomic queue (largest first) and
// solves each one alone, keeping its working matrices in a private slot of
// device memory (L2-resident at these sizes):
//   1.-2. paper form: the Gram products of the bordered blocks [A1 b1] and
//      [A2 b2] on the matrix cores, which give A1^T A1, A2^T A2 and
//      g = A1^T b1 - A2^T b2 (Alg. 1 steps 2-4) in one read of A; correction
//      form: a column pass for g and the non-finite scan, then A1^T A1 (FP64,
//      or FP32 inputs with FP32 accumulation in the mixed form);
//   3. block Gauss-Jordan on [A1^T A1 | A2^T A2 | g] (paper form, giving B, c
//      of Alg. 1) or [A1^T A1 | I] (correction form, giving P), 64-wide blocks,
//      pivot blocks inverted by 16 x 16 blocks (invert64_blk);
//   4. outer steps x_{k+1} = B x_k + c, or x_{k+1} = x_k + P A^T J (b - A x_k)
//      with the residual in FP64 (iterative refinement in the mixed form),
//      with the stop test of the single-problem solver.
// All sums run in a fixed order, so results do not depend on which workgroup
// solves a problem.  The last workgroup to finish resets the queue, so the
// same launch can be replayed (hipGraph) without a host-side reset.
#include "ils_blocks.hpp"
#include "ils_common.hpp"
#include "k_batched.hpp"

namespace ils {

namespace {

constexpr int NT = 256;

struct Smem {
  union {
    struct {
      double T0[kNB][kNB + 1];
      double T1[kNB][kNB + 1];
    } gj;
    struct {
      double As[kNB][kNB + 1];  // As[column][k] of the current 32-row stage
      double Bs[kNB][kNB + 1];
    } g64;
    struct {
      float As[kNB][kNB + 1];
      float Bs[kNB][kNB + 1];
    } g32;
    double vec[2 * kNB * (kNB + 1)];  // iteration phase: t (m), x_k (n)
  } u;
  InvBlk inv;
  double red[2][NT / kWave];
  int id;
};

// One LDS block per workgroup, at file scope so that the out-of-line helper
// functions address it as LDS (ds_* instructions) rather than through
// generic pointers.
__shared__ Smem bsm;

template <typename T>
struct Mma;
template <>
struct Mma<double> {
  typedef v4d acc_t;
  __device__ static acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mma<float> {
  typedef v4f acc_t;
  __device__ static acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <typename T>
__device__ inline T (*stage_a(Smem& s))[kNB + 1];
template <>
__device__ inline double (*stage_a<double>(Smem& s))[kNB + 1] { return s.u.g64.As; }
template <>
__device__ inline float (*stage_a<float>(Smem& s))[kNB + 1] { return s.u.g32.As; }
template <typename T>
__device__ inline T (*stage_b(Smem& s))[kNB + 1];
template <>
__device__ inline double (*stage_b<double>(Smem& s))[kNB + 1] { return s.u.g64.Bs; }
template <>
__device__ inline float (*stage_b<float>(Smem& s))[kNB + 1] { return s.u.g32.Bs; }

__device__ inline double block_sum2(double v, Smem& s, int which) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) s.red[which][w] = v;
  __syncthreads();
  double r = s.red[which][0];
#pragma unroll
  for (int i = 1; i < NT / kWave; ++i) r += s.red[which][i];
  return r;
}

// G = A[0:K, :]^T A[0:K, :] (n x n, full) into W (ldw), one 64 x 64 lower tile
// at a time.  With a border column vb (K entries) the product is that of
// [A vb], whose border row A^T vb goes to gv (n entries).  Each tile streams K in stages of 32 rows: a thread holds 8
// values of each operand panel in flight (one 256-byte column segment per
// half wave per load), then the stage goes through LDS and the next stage's
// loads are issued before the matrix-core work on the current one.  One
// workgroup streams a whole problem, so loads in flight, not bandwidth, set
// the rate; the second workgroup on the CU covers its waits.
template <typename T, int SR>
__device__ __attribute__((noinline)) void wg_gram(const double* A_, int64_t lda, int K, int n, double* W_,
                                                 int64_t ldw, const double* vb_, double* gv_) {
  Smem& s = bsm;
  const auto A = glb(A_);
  const auto W = glb(W_);
  const auto vb = glb(vb_);
  const auto gv = glb(gv_);
  const bool border = vb_ != nullptr;
  typedef typename Mma<T>::acc_t acc_t;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32, lr = lane & 15;
  // SR-row stages (SR / 4 loads per operand per thread; 32 by default: two
  // workgroups share a CU, so registers are scarce and the other workgroup
  // hides latency; the autotuner may pick 16 or 64)
  static_assert(SR == 16 || SR == 32 || SR == 64, "stage rows");
  constexpr int NLD = SR / 4, CG = NT / SR;
  const int lk = t % SR, lc = t / SR;
  const int nt = (n + (border ? 1 : 0) + kNB - 1) / kNB;
  T(*As)[kNB + 1] = stage_a<T>(s);
  T(*Bs)[kNB + 1] = stage_b<T>(s);
  for (int ti = 0; ti < nt; ++ti) {
    for (int tj = 0; tj <= ti; ++tj) {
      const bool diag = ti == tj;
      const auto Ai = A + (int64_t)ti * kNB * lda;
      const auto Aj = A + (int64_t)tj * kNB * lda;
      const int ci = n - ti * kNB, cj = n - tj * kNB;
      acc_t acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = acc_t{};
      T ra[NLD], rb[NLD];
      auto fetch = [&](int k0) {
        const int k = k0 + lk;
        const bool kin = k < K;
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
          const int c = lc + CG * q;
          // column n of the bordered matrix is vb (it can only fall in a
          // diagonal tile's column range when tj < ti, never in Aj's)
          ra[q] = !kin ? (T)0 : c < ci ? (T)Ai[k + (int64_t)c * lda] : (border && c == ci) ? (T)vb[k] : (T)0;
          if (!diag) rb[q] = (kin && c < cj) ? (T)Aj[k + (int64_t)c * lda] : (T)0;
        }
      };
      if (K > 0) fetch(0);
      for (int k0 = 0; k0 < K; k0 += SR) {
        __syncthreads();  // LDS free (previous stage, tile or phase)
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
          As[lc + CG * q][lk] = ra[q];
          if (!diag) Bs[lc + CG * q][lk] = rb[q];
        }
        __syncthreads();
        if (k0 + SR < K) fetch(k0 + SR);
        T(*Bp)[kNB + 1] = diag ? As : Bs;
#pragma unroll
        for (int kk = 0; kk < SR; kk += 4) {
          const int kr = kk + (lane >> 4);
          const T a0 = As[wr + lr][kr], a1 = As[wr + 16 + lr][kr];
          const T b0 = Bp[wc + lr][kr], b1 = Bp[wc + 16 + lr][kr];
          acc[0][0] = Mma<T>::run(a0, b0, acc[0][0]);
          acc[0][1] = Mma<T>::run(a0, b1, acc[0][1]);
          acc[1][0] = Mma<T>::run(a1, b0, acc[1][0]);
          acc[1][1] = Mma<T>::run(a1, b1, acc[1][1]);
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = ti * kNB + wr + a * 16 + Mma<T>::row(lane, v);
            const int j = tj * kNB + wc + c * 16 + lr;
            const double val = (double)acc[a][c][v];
            if (i < n && j < n) {
              W[i + (int64_t)j * ldw] = val;
              if (!diag) W[j + (int64_t)i * ldw] = val;
            } else if (border && i == n && j < n) {
              gv[j] = val;
            }
          }
    }
  }
  __syncthreads();
}

// Block Gauss-Jordan on W = [G | R] (n x ncols), 64-wide blocks, inside one
// workgroup.  Returns false when a pivot block is not positive definite.
__device__ __attribute__((noinline)) bool wg_gauss_jordan(double* W_, int64_t ldw, int n, int ncols) {
  Smem& s = bsm;
  const auto W = glb(W_);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, lr = lane & 15;
  const int hq = (w >> 1) * 32, lq = (w & 1) * 32;
  for (int k0 = 0; k0 < n; k0 += kNB) {
    const int nb = n - k0 < kNB ? n - k0 : kNB;
    __syncthreads();
    {
      double dv[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = t + q * NT, r = e & (kNB - 1), c = e >> 6;
        dv[q] = (r < nb && c < nb) ? W[k0 + r + (int64_t)(k0 + c) * ldw] : (r == c ? 1.0 : 0.0);
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = t + q * NT;
        s.u.gj.T0[e & (kNB - 1)][e >> 6] = dv[q];
      }
    }
    __syncthreads();
    // T0 <- D^{-1} (row-major); T1 serves as the second inversion buffer
    if (!invert64_blk(&s.u.gj.T0[0][0], &s.u.gj.T1[0][0], s.inv)) return false;
    // pivot rows: R = D^{-1} X for every trailing strip (R^T formed so stores run down columns)
    for (int cs = k0 + nb; cs < ncols; cs += kNB) {
      __syncthreads();
      {
        double xv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int e = t + q * NT, lo = e & (kNB - 1), hi = e >> 6;
          xv[q] = (lo < nb && cs + hi < ncols) ? W[k0 + lo + (int64_t)(cs + hi) * ldw] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int e = t + q * NT;
          s.u.gj.T1[e >> 6][e & (kNB - 1)] = xv[q];
        }
      }
      __syncthreads();
      v4d acc[2][2];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < kNB; kk += 4) {
        const int kr = kk + (lane >> 4);
        const double x0 = s.u.gj.T1[hq + lr][kr], x1 = s.u.gj.T1[hq + 16 + lr][kr];
        const double d0 = s.u.gj.T0[lq + lr][kr], d1 = s.u.gj.T0[lq + 16 + lr][kr];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, d0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, d1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, d0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, d1, acc[1][1], 0, 0, 0);
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int c = hq + x * 16 + (lane >> 4) + 4 * v, i = lq + y * 16 + lr;
            if (i < nb && cs + c < ncols) W[k0 + i + (int64_t)(cs + c) * ldw] = acc[x][y][v];
          }
    }
    // other rows: W[I, J] -= W[I, K] R[K, J]
    for (int rs = 0; rs < n; rs += kNB) {
      if (rs == k0) continue;
      __syncthreads();
      {
        double wv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int e = t + q * NT, lo = e & (kNB - 1), hi = e >> 6;
          wv[q] = (rs + lo < n && hi < nb) ? W[rs + lo + (int64_t)(k0 + hi) * ldw] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int e = t + q * NT;
          s.u.gj.T0[e & (kNB - 1)][e >> 6] = wv[q];
        }
      }
      for (int cs = k0 + nb; cs < ncols; cs += kNB) {
        __syncthreads();
        {
          double rv[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int e = t + q * NT, lo = e & (kNB - 1), hi = e >> 6;
            rv[q] = (lo < nb && cs + hi < ncols) ? W[k0 + lo + (int64_t)(cs + hi) * ldw] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int e = t + q * NT;
            s.u.gj.T1[e >> 6][e & (kNB - 1)] = rv[q];
          }
        }
        __syncthreads();
        double cur[2][2][4];
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
          for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int j = hq + a2 * 16 + (lane >> 4) + 4 * v, i = lq + c * 16 + lr;
              cur[a2][c][v] = (rs + i < n && cs + j < ncols) ? W[rs + i + (int64_t)(cs + j) * ldw] : 0.0;
            }
        v4d acc[2][2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < kNB; kk += 4) {
          const int kr = kk + (lane >> 4);
          const double a0 = s.u.gj.T1[hq + lr][kr], a1 = s.u.gj.T1[hq + 16 + lr][kr];
          const double b0 = s.u.gj.T0[lq + lr][kr], b1 = s.u.gj.T0[lq + 16 + lr][kr];
          acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
          for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int j = hq + a2 * 16 + (lane >> 4) + 4 * v, i = lq + c * 16 + lr;
              if (rs + i < n && cs + j < ncols) W[rs + i + (int64_t)(cs + j) * ldw] = cur[a2][c][v] - acc[a2][c][v];
            }
      }
    }
  }
  __syncthreads();
  return true;
}

// t = b - A x (x staged in LDS), then r = A^T J t; t lives in LDS.
constexpr int kXsOff = 4096;  // x_k's offset in the LDS vector area
constexpr int kVsOff = 4608;  // the outer product's vector (n <= 256 entries)
__device__ __attribute__((noinline)) void wg_residual(const double* A_, int64_t lda, int p, int q, int n,
                                                     const double* b_, double* r_) {
  // One pass over A: the workgroup takes blocks of 16 rows; thread
  // (k = t % 16, g = t / 16) holds row k of the block at columns g, g + 16,
  // ... (n <= 256: 16 values), t_k = b_k - (A x)_k is formed with the other 15
  // column groups through LDS, and J_kk t_k A_kc is added to the thread's
  // column sums, which a 16-lane butterfly adds at the end.
  constexpr int R = 16, G = NT / R, PER = 16;
  const auto A = glb(A_);
  const auto b = glb(b_);
  const auto r = glb(r_);
  const double* xs = bsm.u.vec + kXsOff;
  double* red = bsm.u.vec;           // [NT / kWave][R]
  double* tk = bsm.u.vec + 4 * R;    // [R]
  const int m = p + q, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int k = t & (R - 1), g = t / R;
  double acc[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = 0.0;
  for (int i0 = 0; i0 < m; i0 += R) {
    const int i = i0 + k;
    double av[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int c = g + G * u;
      av[u] = (i < m && c < n) ? A[i + (int64_t)c * lda] : 0.0;
    }
    const double bi = (t < R && i < m) ? b[i] : 0.0;
    double sdot = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) sdot = fma(av[u], (g + G * u < n) ? xs[g + G * u] : 0.0, sdot);
    sdot += lane_xor16(sdot);
    sdot += lane_xor32(sdot);
    if (lane < R) red[w * R + k] = sdot;
    __syncthreads();
    if (t < R) {
      const double tot = ((red[t] + red[R + t]) + red[2 * R + t]) + red[3 * R + t];
      double tv = 0.0;
      if (i < m) {
        tv = bi - tot;
        if (i >= p) tv = -tv;  // J = diag(I_p, -I_q)
      }
      tk[t] = tv;
    }
    __syncthreads();
    const double tj = tk[k];
#pragma unroll
    for (int u = 0; u < PER; ++u) acc[u] = fma(tj, av[u], acc[u]);
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const double v = row16_sum(acc[u]);
    const int c = g + G * u;
    if (k == 0 && c < n) r[c] = v;
  }
  __syncthreads();
}

template <typename T, int SR>
__device__ void solve_one(const BatchArgs& a, const BatchProblem& P, double* slot, BatchResult& out) {
  Smem& s = bsm;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int n = (int)P.n, p = (int)P.p, q = (int)P.q, m = p + q;
  const int64_t lda = P.lda, ldw = a.ldw;
  const bool paper = a.form == ILS_FORM_PAPER;
  double* W = slot;
  double* g = slot + a.w_doubles;
  double* xa = g + a.nmax;
  double* xb = xa + a.nmax;
  double* r = xb + a.nmax;
  out.iters = 0;
  out.metric = 0.0;
  // 1. A^T J b and the screen for non-finite input.  Paper form: from the
  // Gram products of the bordered blocks [A1 b1] and [A2 b2], whose border
  // rows hold A1^T b1 and A2^T b2, so A is read once; a non-finite entry of A
  // or b then shows in a Gram diagonal or in g.  Correction form: a column
  // pass (b staged in LDS).
  bool ok = true;
  int nrhs;
  if (paper) {
    // 2. [A1^T A1 | A2^T A2 | g]
    wg_gram<double, SR>(P.A, lda, p, n, W, ldw, P.b, g);
    wg_gram<double, SR>(P.A + p, lda, q, n, W + (int64_t)n * ldw, ldw, P.b + p, xb);
    for (int j = t; j < n; j += NT) {
      const double gj = g[j] - xb[j];
      g[j] = gj;
      W[j + (int64_t)2 * n * ldw] = gj;
      ok &= isfinite(gj) && isfinite(W[j + (int64_t)j * ldw]) && isfinite(W[j + (int64_t)(n + j) * ldw]);
    }
    nrhs = n + 1;
  } else {
    double* bs = s.u.vec;
    for (int i = t; i < m; i += NT) {
      const double bv = glb(P.b)[i];
      bs[i] = bv;
      ok &= isfinite(bv);
    }
    __syncthreads();
    // eight loads of a column in flight, then their products in order
    auto colsum = [&](auto col, int lo, int hi) {
      constexpr int CB = 8;
      double sacc = 0.0;
      for (int i0 = lo + lane; i0 < hi; i0 += CB * kWave) {
        double av[CB];
#pragma unroll
        for (int u = 0; u < CB; ++u) {
          const int i = i0 + u * kWave;
          av[u] = i < hi ? col[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < CB; ++u) {
          const int i = i0 + u * kWave;
          if (i < hi) sacc += av[u] * bs[i];
          ok &= isfinite(av[u]);
        }
      }
      return wave_sum(sacc);
    };
    for (int j = w; j < n; j += NT / kWave) {
      const auto col = glb(P.A) + (int64_t)j * lda;
      const double s1 = colsum(col, 0, p), s2 = colsum(col, p, m);
      if (lane == 0) g[j] = s1 - s2;
    }
    nrhs = n;
  }
  if (__syncthreads_or(!ok)) {
    out.status = ILS_ERR_NONFINITE;
    return;
  }
  double gn2 = 0.0, xr2 = 0.0;
  for (int j = t; j < n; j += NT) gn2 += g[j] * g[j];
  gn2 = block_sum2(gn2, s, 0);
  if (a.stop_rule == ILS_STOP_XREF) {
    for (int j = t; j < n; j += NT) xr2 += glb(P.x_ref)[j] * glb(P.x_ref)[j];
    xr2 = block_sum2(xr2, s, 1);
  }
  if (!paper) {
    // 2. [A1^T A1 | I]
    wg_gram<T, SR>(P.A, lda, p, n, W, ldw, nullptr, nullptr);
    for (int e = t; e < n * n; e += NT) {
      const int i = e % n, j = e / n;
      W[i + (int64_t)(n + j) * ldw] = (i == j) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  // 3. elimination
  if (!wg_gauss_jordan(W, ldw, n, n + nrhs)) {
    out.status = ILS_ERR_NOT_SPD;
    return;
  }
  const double* M = W + (int64_t)n * ldw;  // B (paper) or P (correction)
  const double* c = W + (int64_t)2 * n * ldw;
  // 4. outer steps
  double* xs = s.u.vec + kXsOff;  // n entries (x_k staged for the residual)
  double* vs = s.u.vec + kVsOff;  // n entries (the vector of the outer step's product)
  for (int j = t; j < n; j += NT) xa[j] = P.x0 ? glb(P.x0)[j] : 0.0;
  __syncthreads();
  double* xk = xa;
  double* xn = xb;
  const bool need_r = !paper || a.stop_rule == ILS_STOP_RR;
  int status = ILS_OK;
  int64_t k = 0;
  double metric = 0.0;
  // the test on x_k first when it does not need r_k (relative error, fixed
  // count), so the iterate that ends the loop costs no pass over A; and
  // r_0 = A^T J b at x_0 = 0 is the column pass's g
  const bool r_first = a.stop_rule == ILS_STOP_RR;
  for (;; ++k) {
    auto residual = [&]() {
      if (!need_r) return;
      if (k == 0 && !P.x0 && !paper) {
        for (int j = t; j < n; j += NT) r[j] = g[j];
        __syncthreads();
        return;
      }
      for (int j = t; j < n; j += NT) xs[j] = xk[j];
      __syncthreads();
      wg_residual(P.A, lda, p, q, n, P.b, r);
    };
    if (r_first) residual();
    double mp = 0.0;
    for (int j = t; j < n; j += NT) {
      if (a.stop_rule == ILS_STOP_XREF) {
        const double d = xk[j] - glb(P.x_ref)[j];
        mp += d * d;
      } else if (a.stop_rule == ILS_STOP_RR) {
        mp += r[j] * r[j];
      }
    }
    mp = block_sum2(mp, s, (int)(k & 1));
    metric = a.stop_rule == ILS_STOP_XREF ? sqrt(mp) / sqrt(xr2) : mp / gn2;
    if (a.stop_rule != ILS_STOP_FIXED && metric < a.tol) break;
    if (k == a.max_outer) {
      status = a.stop_rule == ILS_STOP_FIXED ? ILS_OK : ILS_ERR_NO_CONVERGENCE;
      break;
    }
    if (!r_first) residual();
    bool bad = false;
    {
      const double* v = paper ? xk : r;
      for (int j = t; j < n; j += NT) vs[j] = v[j];
    }
    __syncthreads();
    for (int i = t; i < n; i += NT) {
      // sixteen loads of the row in flight, then the products in order
      double acc = 0.0;
      for (int j0 = 0; j0 < n; j0 += 16) {
        double mv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) mv[u] = M[i + (int64_t)(j0 + u < n ? j0 + u : n - 1) * ldw];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (j0 + u < n) acc += mv[u] * vs[j0 + u];
      }
      const double xi = paper ? acc + c[i] : xk[i] + acc;
      xn[i] = xi;
      bad |= !isfinite(xi);
    }
    bad = __syncthreads_or(bad);
    double* tmp = xk;
    xk = xn;
    xn = tmp;
    if (bad) {
      status = ILS_ERR_NONFINITE;
      ++k;
      break;
    }
  }
  for (int j = t; j < n; j += NT) glb(P.x)[j] = xk[j];
  out.status = status;
  out.iters = k;
  out.metric = metric;
}

// Two workgroups per CU: the register budget is cut to fit them (the helper
// functions spill a little at entry), and each hides the other's latency.
template <typename T, int SR>
__global__ __launch_bounds__(NT, 2) void k_batched(BatchArgs a) {
  Smem& s = bsm;
  double* slot = a.work + (int64_t)blockIdx.x * a.slot_doubles;
  for (;;) {
    if (threadIdx.x == 0) s.id = (int)atomicAdd(&a.queue[0], 1u);
    __syncthreads();
    const int id = s.id;
    __syncthreads();
    if (id >= a.count) break;
    const int idx = a.order[id];
    BatchResult res;
    res.status = ILS_OK;
    solve_one<T, SR>(a, a.probs[idx], slot, res);
    if (threadIdx.x == 0) a.res[idx] = res;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&a.queue[1], 1u) == gridDim.x - 1) {
      a.queue[0] = 0;
      a.queue[1] = 0;
      __threadfence();
    }
  }
}

}  // namespace

template <int SR>
static void launch_sr(hipStream_t s, const BatchArgs& a, int workgroups) {
  if (a.precision == ILS_PREC_MIXED)
    hipLaunchKernelGGL((k_batched<float, SR>), dim3(workgroups), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_batched<double, SR>), dim3(workgroups), dim3(NT), 0, s, a);
}

void launch_batched(hipStream_t s, const BatchArgs& a, int workgroups, int stage_rows) {
  if (stage_rows == 16)
    launch_sr<16>(s, a, workgroups);
  else if (stage_rows == 64)
    launch_sr<64>(s, a, workgroups);
  else
    launch_sr<32>(s, a, workgroups);
}

}  // namespace ils
