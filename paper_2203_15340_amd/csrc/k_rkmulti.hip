// k_rkmulti.hip -- SP-RK-RGS inner steps (Alg. 2 steps 8-11) for up to
// kMR right-hand sides at once that share one index stream.
//
// The column draws j1(t), j2(t) depend only on the column norms of A1, so
// every right-hand side of a family that shares A can follow the same
// stream: each keeps its own w_r, s_r = w_r - A1 z_r and z_r, and each
// follows exactly the iterates it would follow alone.  A block of kRB steps
// gathers u_t = A1_(j1(t)), v_t = A1_(j2(t)) once for all of them, so the
// block's inner products are one product [U V]^T [U V W S] over the rows of
// A1 (the gathered columns against themselves and against every w_r, s_r:
// a GEMM where a single right-hand side has a GEMV), and the update is
// W += U Gamma, S += U Gamma - V Delta with a coefficient column per
// right-hand side.  The scalar recurrences of each right-hand side are those
// of the single-right-hand-side kernel (k_rkblock.hip), one wave each.
// A right-hand side whose inner loop is over (or whose outer loop is over)
// takes zero coefficients: its w, s and z no longer change.
#include "ils_common.hpp"
#include "k_rand.hpp"

namespace ils {

constexpr int kMRB = 32;               // steps per block
constexpr int kMRX = 2 * kMRB;         // gathered columns u_0.., v_0..
constexpr int kMRY = kMRX + 2 * kMR;   // + w_r, s_r of every right-hand side
constexpr int kMRS = 128;              // rows of a slice held in LDS at once
constexpr int kMRL = kMRS + 1;         // LDS row stride
constexpr int kMRWcol = kMRX;          // first w column
constexpr int kMRScol = kMRX + kMR;    // first s column

__device__ inline const double* mr_col(const double* A1, int64_t lda, const int* j1, const int* j2, int bt, int c) {
  if (c < kMRB) return c < bt ? A1 + (int64_t)j1[c] * lda : nullptr;
  return c - kMRB < bt ? A1 + (int64_t)j2[c - kMRB] * lda : nullptr;
}

// Per row slice: the previous block's update of W, S, then this block's
// partial of C = [U V]^T [U V W S] (rows of u against U and W, rows of v
// against U, V and S: the entries the recurrences read).
__global__ __launch_bounds__(256) void k_rkbm_step(const double* __restrict__ A1, int64_t lda, int64_t p,
                                                   int R, const int* __restrict__ pj1,
                                                   const int* __restrict__ pj2, int pbt,
                                                   const double* __restrict__ coef,
                                                   const int* __restrict__ j1, const int* __restrict__ j2,
                                                   int bt, double* __restrict__ W, double* __restrict__ S,
                                                   int64_t ldw, int64_t slice_rows, double* __restrict__ part) {
  __shared__ double Ms[kMRY][kMRL];
  __shared__ double cf[kMR * kMRX];  // cf[r * kMRX + t]: gamma_t (t < kMRB), delta (t >= kMRB)
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, lr = lane & 15;
  const int lk = t & 15, cg = t >> 4;
  const double* ps[4];
  const double* ns[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ps[q] = mr_col(A1, lda, pj1, pj2, pbt, cg + 16 * q);
    ns[q] = mr_col(A1, lda, j1, j2, bt, cg + 16 * q);
  }
  for (int e = t; e < kMR * kMRX; e += 256) cf[e] = (pbt > 0 && e / kMRX < R) ? coef[e] : 0.0;
  v4d acc[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) acc[c] = v4d{};
  const int64_t s0 = (int64_t)blockIdx.x * slice_rows;
  const int64_t s1 = s0 + slice_rows < p ? s0 + slice_rows : p;
  for (int64_t r0 = s0; r0 < s1; r0 += kMRS) {
    const int nr = (int)(s1 - r0 < kMRS ? s1 - r0 : kMRS);
    const int nr16 = (nr + 15) & ~15;
    double pv[4][kMRS / 16], nv[4][kMRS / 16];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int rr = 0; rr < kMRS / 16; ++rr) {
        const int k = lk + 16 * rr;
        pv[q][rr] = (ps[q] && k < nr) ? ps[q][r0 + k] : 0.0;
        nv[q][rr] = (ns[q] && k < nr) ? ns[q][r0 + k] : 0.0;
      }
    __syncthreads();  // the previous chunk's reads of Ms are done
    // W, S of the chunk into their Ms columns (zero for unused right-hand sides)
    for (int e = t; e < 2 * kMR * kMRS; e += 256) {
      const int col = e / kMRS, i = e % kMRS, r = col % kMR;
      const bool isw = col < kMR;
      double v = 0.0;
      if (r < R && i < nr) v = isw ? W[r0 + i + r * ldw] : S[r0 + i + r * ldw];
      Ms[(isw ? kMRWcol : kMRScol) + r][i] = v;
    }
    if (pbt > 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int rr = 0; rr < kMRS / 16; ++rr) Ms[cg + 16 * q][lk + 16 * rr] = pv[q][rr];
      __syncthreads();
      // row i, right-hand sides r = hr, hr + 2, ...: dw = sum gamma u(i),
      // dv = sum delta v(i), each as two chains of 16 in column order
      const int i = t & (kMRS - 1), hr = t >> 7;
      if (i < nr) {
        for (int r = hr; r < R; r += 2) {
          const double* cr = cf + r * kMRX;
          double h0 = 0.0, h1 = 0.0, d0 = 0.0, d1 = 0.0;
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            h0 = fma(cr[u], Ms[u][i], h0);
            d0 = fma(cr[kMRB + u], Ms[kMRB + u][i], d0);
          }
#pragma unroll
          for (int u = 16; u < 32; ++u) {
            h1 = fma(cr[u], Ms[u][i], h1);
            d1 = fma(cr[kMRB + u], Ms[kMRB + u][i], d1);
          }
          const double dw = h0 + h1, dv = d0 + d1;
          const double wn = Ms[kMRWcol + r][i] + dw;
          const double sn = Ms[kMRScol + r][i] + (dw - dv);
          Ms[kMRWcol + r][i] = wn;
          Ms[kMRScol + r][i] = sn;
          W[r0 + i + r * ldw] = wn;
          S[r0 + i + r * ldw] = sn;
        }
      }
      __syncthreads();  // the update's reads of the gathered columns are done
    }
    if (bt == 0) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int rr = 0; rr < kMRS / 16; ++rr) Ms[cg + 16 * q][lk + 16 * rr] = nv[q][rr];
    __syncthreads();
    // waves 0, 1: u rows against U (blocks 0, 1) and W (block 4); waves 2, 3:
    // v rows against U, V (blocks 0-3) and S (block 5)
    for (int kk = 0; kk < nr16; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double a = Ms[16 * wv + lr][kr];
#pragma unroll
      for (int c = 0; c < 6; ++c)
        if (wv >= 2 ? c != 4 : (c < 2 || c == 4))
          acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ms[16 * c + lr][kr], acc[c], 0, 0, 0);
    }
  }
  if (bt == 0) return;
  double* P = part + (int64_t)blockIdx.x * (kMRX * kMRY);
#pragma unroll
  for (int c = 0; c < 6; ++c)
    if (wv >= 2 ? c != 4 : (c < 2 || c == 4))
#pragma unroll
      for (int v = 0; v < 4; ++v) P[(16 * wv + (lane >> 4) + 4 * v) * kMRY + 16 * c + lr] = acc[c][v];
}

__device__ inline bool mr_needed(int e) {
  const int r = e / kMRY, c = e % kMRY;
  if (r < kMRB) return c < kMRB || (c >= kMRWcol && c < kMRWcol + kMR);
  return c < kMRX || c >= kMRScol;
}

__device__ inline double mr_lane(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Right-hand side r's two lower-triangular solves of size bt (the recurrences
// of the single-right-hand-side kernel), one wave; frozen: zero coefficients.
__device__ __attribute__((always_inline)) inline void rkbm_recur_wave(const double* C, int bt, int r, bool frozen,
                                                                      const int* __restrict__ j1,
                                                                      const int* __restrict__ j2,
                                                                      const double* __restrict__ tgt,
                                                                      const double* __restrict__ cn,
                                                                      double* __restrict__ z,
                                                                      double* __restrict__ coef) {
  const int lane = threadIdx.x & 63;
  double* cr = coef + r * kMRX;
  if (frozen) {
    cr[lane] = 0.0;
    return;
  }
  const int tau = lane < kMRB ? lane : kMRB - 1;
  const bool live = lane < bt;
  const int a = live ? j1[lane] : 0, b = live ? j2[lane] : -1;
  const double rcg = live ? 1.0 / cn[a] : 0.0;
  const double rcd = live ? 1.0 / cn[b] : 0.0;
  auto ld = [&](int e) { return __hip_atomic_load(C + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
  double rg = live ? tgt[a] - ld(tau * kMRY + kMRWcol + r) : 0.0;
  double rd = live ? ld((kMRB + tau) * kMRY + kMRScol + r) : 0.0;
  double uu[kMRB], vu[kMRB], vv[kMRB];
#pragma unroll
  for (int k = 0; k < kMRB; ++k) {
    uu[k] = ld(tau * kMRY + k);
    vu[k] = ld((kMRB + tau) * kMRY + k);
    vv[k] = ld((kMRB + tau) * kMRY + kMRB + k);
  }
  double gam = 0.0, del = 0.0;
#pragma unroll
  for (int t = 0; t < kMRB; ++t) {
    if (t < bt) {
      const double g = mr_lane(rg * rcg, t);
      if (lane == t) gam = g;
      if (lane > t) rg = fma(-uu[t], g, rg);
      if (lane >= t) rd = fma(vu[t], g, rd);
    }
  }
#pragma unroll
  for (int t = 0; t < kMRB; ++t) {
    if (t < bt) {
      const double d = mr_lane(rd * rcd, t);
      if (lane == t) del = d;
      if (lane > t) rd = fma(-vv[t], d, rd);
    }
  }
  if (lane < kMRB) {
    cr[lane] = live ? gam : 0.0;
    cr[kMRB + lane] = live ? del : 0.0;
  }
  bool first = live;
  double sum = 0.0;
  for (int u = 0; u < bt; ++u) {
    const int bu = __builtin_amdgcn_readlane(b, u);
    const double du = mr_lane(del, u);
    if (bu == b) {
      if (u < lane) first = false;
      else sum += du;
    }
  }
  if (first) z[b] += sum;
}

// C = sum of the slices' partials in slice order (deterministic); the last
// workgroup to arrive runs every right-hand side's recurrences (wave w takes
// r = w, w + 4, ...).
constexpr int kMRedE = 32;
constexpr int kMRedG = 8;
constexpr int kMRedDepth = 32;

struct RkmClose {
  const double* part;
  int nslices;
  double* C;
  unsigned* arrive;
  int bt, R;
  const int* j1;
  const int* j2;
  const double* tgt;  // n x R (ldt)
  int64_t ldt;
  const double* cn;
  double* Z;          // n x R (ldz)
  int64_t ldz;
  double* coef;       // kMRX x R
  const int* frozen;  // R flags (inner loop over, or column retired)
};

__global__ __launch_bounds__(256) void k_rkbm_close(RkmClose a) {
  __shared__ double red[kMRedG][kMRedE];
  __shared__ int is_last;
  const int le = threadIdx.x & (kMRedE - 1), g = threadIdx.x / kMRedE;
  const int e = blockIdx.x * kMRedE + le;
  double acc = 0.0;
  if (e < kMRX * kMRY && mr_needed(e)) {
    for (int s0 = g; s0 < a.nslices; s0 += kMRedG * kMRedDepth) {
      double v[kMRedDepth];
#pragma unroll
      for (int u = 0; u < kMRedDepth; ++u) {
        const int sl = s0 + kMRedG * u;
        v[u] = sl < a.nslices ? a.part[(int64_t)sl * (kMRX * kMRY) + e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kMRedDepth; ++u) acc += v[u];
    }
  }
  red[g][le] = acc;
  __syncthreads();
  // C goes to the last workgroup through device-scope stores and loads, as
  // in the single-right-hand-side close: the writing wave waits for its
  // stores, then counts (no device-scope fence per workgroup)
  if (threadIdx.x < kMRedE && e < kMRX * kMRY) {
    double tot = red[0][le];
#pragma unroll
    for (int u = 1; u < kMRedG; ++u) tot += red[u][le];
    __hip_atomic_store(a.C + e, tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __asm__ __volatile__("" ::: "memory");
  if (threadIdx.x == 0) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): wave 0's stores of C have completed
    is_last = __hip_atomic_fetch_add(a.arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last) return;
  const int w = threadIdx.x >> 6;
  for (int r = w; r < a.R; r += 4) {
    const bool frozen = *(volatile const int*)(a.frozen + r) != 0;
    rkbm_recur_wave(a.C, a.bt, r, frozen, a.j1, a.j2, a.tgt + r * a.ldt, a.cn, a.Z + r * a.ldz, a.coef);
  }
  __syncthreads();
  if (threadIdx.x == 0) *a.arrive = 0;
}

size_t rk_multi_scratch(int64_t p) {
  const int64_t rows = rk_block_slice_rows(p);
  const int64_t nsl = (p + rows - 1) / rows;
  return (size_t)nsl * kMRX * kMRY + (size_t)kMRX * kMRY + (size_t)kMR * kMRX;
}

void launch_rk_multi_blocks(hipStream_t st, const double* A1, int64_t lda, int64_t p, int R, const double* tgt,
                            int64_t ldt, const double* cn, const int* j1, const int* j2, int64_t count,
                            double* W, double* S, int64_t ldw, double* Z, int64_t ldz, const int* frozen,
                            double* scratch, unsigned* arrive) {
  if (count <= 0 || R <= 0) return;
  const int64_t rows = rk_block_slice_rows(p);
  const int nsl = (int)((p + rows - 1) / rows);
  double* part = scratch;
  double* C = scratch + (int64_t)nsl * kMRX * kMRY;
  double* coef = C + kMRX * kMRY;
  int pbt = 0;
  int64_t pt0 = 0;
  for (int64_t t0 = 0;; t0 += kMRB) {
    const int64_t left = count - t0 > 0 ? count - t0 : 0;
    const int bt = (int)(left < kMRB ? left : kMRB);
    if (bt == 0 && pbt == 0) break;
    hipLaunchKernelGGL(k_rkbm_step, dim3((unsigned)nsl), dim3(256), 0, st, A1, lda, p, R, j1 + pt0, j2 + pt0, pbt,
                       (const double*)coef, j1 + t0, j2 + t0, bt, W, S, ldw, rows, part);
    if (bt == 0) break;
    RkmClose c;
    c.part = part;
    c.nslices = nsl;
    c.C = C;
    c.arrive = arrive;
    c.bt = bt;
    c.R = R;
    c.j1 = j1 + t0;
    c.j2 = j2 + t0;
    c.tgt = tgt;
    c.ldt = ldt;
    c.cn = cn;
    c.Z = Z;
    c.ldz = ldz;
    c.coef = coef;
    c.frozen = frozen;
    hipLaunchKernelGGL(k_rkbm_close, dim3((kMRX * kMRY + kMRedE - 1) / kMRedE), dim3(256), 0, st, c);
    pbt = bt;
    pt0 = t0;
  }
}

// Inner stop test per right-hand side: res_r = tgt_r - AtV_r (AtV = A1^T (W - S)),
// frozen_r = 1 when ||res_r||^2 <= itol2 ||tgt_r||^2.  One workgroup per
// right-hand side; a frozen one is left as it is.
__global__ __launch_bounds__(256) void k_rkm_check(int64_t n, const double* __restrict__ tgt, int64_t ldt,
                                                   const double* __restrict__ AtV, int64_t lda_tv,
                                                   const double* __restrict__ tn2, double itol2,
                                                   int* __restrict__ frozen) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  if (frozen[r]) return;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    const double d = tgt[j + r * ldt] - AtV[j + r * lda_tv];
    s += d * d;
  }
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0 && s <= itol2 * tn2[r]) frozen[r] = 1;
}

__global__ void k_wminus_s(int64_t p, int R, const double* __restrict__ W, const double* __restrict__ S, int64_t ldw,
                           double* __restrict__ V) {
  const int64_t total = p * R;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t r = e / p, i = e - r * p;
    V[e] = W[i + r * ldw] - S[i + r * ldw];
  }
}

void launch_rkm_check(hipStream_t st, const double* A1, int64_t lda, int64_t p, int64_t n, int R, const double* W,
                      const double* S, int64_t ldw, double* V, double* AtV, const double* tgt, int64_t ldt,
                      const double* tn2, double itol2, int* frozen) {
  int64_t blocks = (p * R + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_wminus_s, dim3((unsigned)blocks), dim3(256), 0, st, p, R, W, S, ldw, V);
  GemmTnArgs g = {};
  g.M = n;
  g.N = R;
  g.K = p;
  g.X = A1;
  g.ldx = lda;
  g.Y = V;
  g.ldy = p;
  g.kneg = p;
  g.alpha = 1.0;
  g.beta = 0.0;
  g.C = AtV;
  g.ldc = n;
  launch_gemm_tn(st, g);
  hipLaunchKernelGGL(k_rkm_check, dim3((unsigned)R), dim3(256), 0, st, n, tgt, ldt, (const double*)AtV, n, tn2,
                     itol2, frozen);
}

}  // namespace ils
