// k_mlp.hip -- BF16 kernels of the warm-start network: matrix products on
// the gfx950 matrix cores (bf16 inputs, FP32 accumulation), the loss and bias
// gradients, Adam on FP32 master weights, and input/target standardisation.
//
// The network maps a standardised row sample of b to a standardised estimate
// of x, used as the initial value of the SP iteration (Alg. 1 accepts any
// x0, Thm. 2.1).  theta = [W1, b1, W2, b2, W3, b3], W_l (d_l x d_{l-1})
// row-major.  Activations are column-major, one sample per column.
#include "ils_common.hpp"
#include "k_mlp.hpp"

namespace ils {


__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
// float -> bfloat16, round to nearest even (NaN stays NaN)
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ------------------------------------------------------------------ GEMM
// C (M x N) = op(A) op(B), K-sum in FP32 on gfx950's v_mfma_f32_16x16x32_bf16
// (8 bf16 per lane per operand: lanes 16g..16g+15 hold k = 8g..8g+7 of their
// row or column, so one 16-byte LDS read feeds a whole 32-deep stage).
//   TA = 0: A is M x K column-major, element (i, k) at A[i + k lda]
//   TA = 1: A is stored K x M,       element (i, k) at A[k + i lda]
//   TB = 0: B is K x N column-major, element (k, j) at B[k + j ldb]
//   TB = 1: B is stored N x K,       element (k, j) at B[j + k ldb]
// Workgroup = 64 x 64 tile of C, four waves of 32 x 32.  Each stage moves a
// 64 x 32 panel of both operands into LDS with k contiguous (the order the
// matrix-core operands are read in); panels whose source is k-contiguous
// move as 16-byte vectors, the others are transposed on the way in.
constexpr int kBT = 64;       // tile edge
constexpr int kBK = 32;       // k per stage
constexpr int kBLd = kBK + 8; // padded LDS row (bf16 elements): 80 bytes, rows stay 16-byte aligned

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Load this thread's 8 elements of the 64 x 32 panel (operand rows
// [r0, r0 + 64), k in [k0, k0 + 32)); `rows` bounds the operand's row index
// (i of A, j of B), KCONTIG tells the storage order.  Out of range -> 0.
template <bool KCONTIG>
__device__ inline void panel_fetch(const uint16_t* __restrict__ X, int64_t ld, int64_t rows, int64_t K,
                                   int64_t r0, int64_t k0, int t, uint16_t (&v)[8]) {
  if (KCONTIG) {
    // thread -> row t/4, k segment (t%4)*8
    const int64_t r = r0 + (t >> 2), k = k0 + (t & 3) * 8;
    const uint16_t* src = X + k + r * ld;
    if (r < rows && k + 8 <= K && (((uintptr_t)src) & 15) == 0) {
      const uint4 q = *(const uint4*)src;
      v[0] = q.x & 0xffff; v[1] = q.x >> 16; v[2] = q.y & 0xffff; v[3] = q.y >> 16;
      v[4] = q.z & 0xffff; v[5] = q.z >> 16; v[6] = q.w & 0xffff; v[7] = q.w >> 16;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (r < rows && k + e < K) ? src[e] : (uint16_t)0;
    }
  } else {
    // thread -> k t/8, row segment (t%8)*8
    const int64_t k = k0 + (t >> 3), r = r0 + (t & 7) * 8;
    const uint16_t* src = X + r + k * ld;
    if (k < K && r + 8 <= rows && (((uintptr_t)src) & 15) == 0) {
      const uint4 q = *(const uint4*)src;
      v[0] = q.x & 0xffff; v[1] = q.x >> 16; v[2] = q.y & 0xffff; v[3] = q.y >> 16;
      v[4] = q.z & 0xffff; v[5] = q.z >> 16; v[6] = q.w & 0xffff; v[7] = q.w >> 16;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (k < K && r + e < rows) ? src[e] : (uint16_t)0;
    }
  }
}

template <bool KCONTIG>
__device__ inline void panel_stash(uint16_t (*S)[kBLd], int t, const uint16_t (&v)[8]) {
  if (KCONTIG) {
    const int r = t >> 2, k = (t & 3) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) S[r][k + e] = v[e];
  } else {
    const int k = t >> 3, r = (t & 7) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) S[r + e][k] = v[e];
  }
}

template <int TA, int TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm_bf16(MlpGemmArgs g) {
  __shared__ __align__(16) uint16_t As[kBT][kBLd];
  __shared__ __align__(16) uint16_t Bs[kBT][kBLd];
  const int64_t mt = (g.M + kBT - 1) / kBT;
  const int64_t i0 = (blockIdx.x % mt) * kBT, j0 = (blockIdx.x / mt) * kBT;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int lr = lane & 15, lq = lane >> 4;
  v4f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = v4f{};
  uint16_t va[8], vb[8];
  panel_fetch<TA == 1>(g.A, g.lda, g.M, g.K, i0, 0, t, va);
  panel_fetch<TB == 0>(g.B, g.ldb, g.N, g.K, j0, 0, t, vb);
  for (int64_t k0 = 0; k0 < g.K; k0 += kBK) {
    panel_stash<TA == 1>(As, t, va);
    panel_stash<TB == 0>(Bs, t, vb);
    __syncthreads();
    if (k0 + kBK < g.K) {
      panel_fetch<TA == 1>(g.A, g.lda, g.M, g.K, i0, k0 + kBK, t, va);
      panel_fetch<TB == 0>(g.B, g.ldb, g.N, g.K, j0, k0 + kBK, t, vb);
    }
    static_assert(kBK == 32, "one 16x16x32 step per stage");
    {
      v8bf fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) fa[a] = *(const v8bf*)&As[wr + a * 16 + lr][8 * lq];
#pragma unroll
      for (int c = 0; c < 2; ++c) fb[c] = *(const v8bf*)&Bs[wc + c * 16 + lr][8 * lq];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[c], acc[a][c], 0, 0, 0);
    }
    __syncthreads();
  }
  // output element v of a lane sits at row 4*(lane/16) + v, column lane%16
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int64_t j = j0 + wc + c * 16 + lr;
    if (j >= g.N) continue;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + wr + a * 16 + 4 * lq + v;
        if (i >= g.M) continue;
        const float s = acc[a][c][v];
        if (EPI == kEpiBiasReluBf16) {
          const float z = s + g.bias[i];
          g.Cb[i + j * g.ldc] = f2bf(z > 0.0f ? z : 0.0f);
        } else if (EPI == kEpiBiasF32) {
          g.Cf[i + j * g.ldc] = s + g.bias[i];
        } else if (EPI == kEpiMaskF32) {
          g.Cf[i + j * g.ldc] = g.mask[i + j * g.ldmask] != 0 ? s : 0.0f;  // relu' from h > 0
        } else {
          g.Cf[i * g.csi + j * g.csj] = s;
        }
      }
  }
}

template <int TA, int TB, int EPI>
static void gemm_go(hipStream_t s, const MlpGemmArgs& g) {
  const int64_t tiles = ((g.M + kBT - 1) / kBT) * ((g.N + kBT - 1) / kBT);
  hipLaunchKernelGGL((k_gemm_bf16<TA, TB, EPI>), dim3((unsigned)tiles), dim3(256), 0, s, g);
}

void launch_mlp_gemm(hipStream_t s, int ta, int tb, int epi, const MlpGemmArgs& g) {
  if (g.M <= 0 || g.N <= 0) return;
  if (ta == 1 && tb == 0 && epi == kEpiBiasReluBf16) gemm_go<1, 0, kEpiBiasReluBf16>(s, g);
  else if (ta == 1 && tb == 0 && epi == kEpiBiasF32) gemm_go<1, 0, kEpiBiasF32>(s, g);
  else if (ta == 0 && tb == 0 && epi == kEpiMaskF32) gemm_go<0, 0, kEpiMaskF32>(s, g);
  else if (ta == 0 && tb == 1 && epi == kEpiStoreF32) gemm_go<0, 1, kEpiStoreF32>(s, g);
  else if (ta == 1 && tb == 0 && epi == kEpiStoreF32) gemm_go<1, 0, kEpiStoreF32>(s, g);
  else if (ta == 0 && tb == 0 && epi == kEpiStoreF32) gemm_go<0, 0, kEpiStoreF32>(s, g);
}

// ------------------------------------------------------------------ elementwise
// float -> bf16 copy (weights after an update, inputs of the check entry points)
__global__ void k_f2bf(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = f2bf(x[i]);
}

void launch_f2bf(hipStream_t s, int64_t n, const float* x, uint16_t* y) {
  if (n <= 0) return;
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_f2bf, dim3((unsigned)b), dim3(256), 0, s, n, x, y);
}

// Output layer: dY = 2 (y - t) / (N d3) (FP32 and bf16), bias gradient
// db3[i] = sum_s dY[i, s], and per-row loss sums.  Workgroup = 64 rows x 16
// waves; wave w takes samples w, w + 16, ... (coalesced 64-row segments) and
// the 16 partial sums are added in wave order.
constexpr int kRowWaves = 16;

__global__ __launch_bounds__(64 * kRowWaves) void k_mlp_outgrad(int64_t d3, int64_t N, const float* __restrict__ Y,
                                                               const float* __restrict__ T,
                                                               uint16_t* __restrict__ dYb, float* __restrict__ db,
                                                               double* __restrict__ loss_rows) {
  __shared__ float rb[kRowWaves][64];
  __shared__ double rl[kRowWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const float sc = 2.0f / (float)((double)N * (double)d3);
  float sb = 0.0f;
  double sl = 0.0;
  if (i < d3) {
    for (int64_t s = w; s < N; s += kRowWaves) {
      const float e = Y[i + s * d3] - T[i + s * d3];
      const float dy = sc * e;
      dYb[i + s * d3] = f2bf(dy);
      sb += dy;
      sl += (double)e * (double)e;
    }
  }
  rb[w][lane] = sb;
  rl[w][lane] = sl;
  __syncthreads();
  if (w == 0 && i < d3) {
    float tb = 0.0f;
    double tl = 0.0;
    for (int k = 0; k < kRowWaves; ++k) {
      tb += rb[k][lane];
      tl += rl[k][lane];
    }
    db[i] = tb;
    loss_rows[i] = tl;
  }
}

// loss = sum(loss_rows) / (N d3), one workgroup
__global__ __launch_bounds__(256) void k_mlp_loss(int64_t d3, int64_t N, const double* __restrict__ loss_rows,
                                                  double* __restrict__ out) {
  __shared__ double red[4];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < d3; i += 256) a += loss_rows[i];
  a = block_sum<256>(a, red);
  if (threadIdx.x == 0) *out = a / ((double)N * (double)d3);
}

void launch_mlp_outgrad(hipStream_t s, int64_t d3, int64_t N, const float* Y, const float* T, uint16_t* dYb,
                        float* db, double* loss_rows, double* loss) {
  hipLaunchKernelGGL(k_mlp_outgrad, dim3((unsigned)((d3 + 63) / 64)), dim3(64 * kRowWaves), 0, s, d3, N, Y, T,
                     dYb, db, loss_rows);
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s, d3, N, (const double*)loss_rows, loss);
}

// Hidden layer: db[i] = sum_s dZ[i, s] and dZ -> bf16, same layout as above.
__global__ __launch_bounds__(64 * kRowWaves) void k_mlp_rowsum(int64_t d, int64_t N, const float* __restrict__ dZ,
                                                              uint16_t* __restrict__ dZb, float* __restrict__ db) {
  __shared__ float rb[kRowWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  float sb = 0.0f;
  if (i < d) {
    for (int64_t s = w; s < N; s += kRowWaves) {
      const float v = dZ[i + s * d];
      dZb[i + s * d] = f2bf(v);
      sb += v;
    }
  }
  rb[w][lane] = sb;
  __syncthreads();
  if (w == 0 && i < d) {
    float tb = 0.0f;
    for (int k = 0; k < kRowWaves; ++k) tb += rb[k][lane];
    db[i] = tb;
  }
}

void launch_mlp_rowsum(hipStream_t s, int64_t d, int64_t N, const float* dZ, uint16_t* dZb, float* db) {
  hipLaunchKernelGGL(k_mlp_rowsum, dim3((unsigned)((d + 63) / 64)), dim3(64 * kRowWaves), 0, s, d, N, dZ, dZb, db);
}

// Adam (Kingma & Ba 2015) on the FP32 master copy, then the bf16 copy used by
// the products.  c1 = 1 - beta1^t, c2 = 1 - beta2^t; the host passes
// 1 - beta1 and 1 - beta2 rounded from double (1.0f - 0.999f is off by 1e-5).
__global__ void k_adam(int64_t n, float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, uint16_t* __restrict__ wb, AdamArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = a.b1 * m[i] + a.omb1 * gi;
    const float vi = a.b2 * v[i] + a.omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
  }
}

void launch_adam(hipStream_t s, int64_t n, float* w, float* m, float* v, const float* g, uint16_t* wb,
                 const AdamArgs& a) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)b), dim3(256), 0, s, n, w, m, v, g, wb, a);
}

// Initial weights: W_l ~ N(0, 2 / d_{l-1}) (He), biases 0.  Normal draws by
// Box-Muller from Philox4x64-10 with counter (element, 0, 0, 0), key (seed, tag).
__global__ void k_mlp_init(int64_t n, const int64_t* __restrict__ seg, float* __restrict__ w, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    // seg: [offW1, offb1, offW2, offb2, offW3, offb3, end] and fan-ins at [7..9]
    int l = 0;
    while (l < 2 && i >= seg[2 * l + 2]) ++l;
    if (i >= seg[2 * l + 1]) {
      w[i] = 0.0f;
      continue;
    }
    uint64_t r[4];
    philox4x64_10((uint64_t)i, 0, 0, 0, seed, 0x4D4C50ull, r);
    const double u1 = ((double)(r[0] >> 11) + 1.0) * (1.0 / 9007199254740992.0);  // (0, 1]
    const double u2 = (double)(r[1] >> 11) * (1.0 / 9007199254740992.0);
    const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    w[i] = (float)(z * sqrt(2.0 / (double)seg[7 + l]));
  }
}

void launch_mlp_init(hipStream_t s, int64_t n, const int64_t* seg, float* w, uint64_t seed) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_mlp_init, dim3((unsigned)b), dim3(256), 0, s, n, seg, w, seed);
}

// Feature statistics over N samples: feature r of sample s is
// X[rows[r] + s ldx] (rows == null: row r).  Partial FP64 sums per
// (feature, chunk of samples), then mean and standard deviation.
constexpr int kStatChunks = 64;

__global__ __launch_bounds__(256) void k_stats_part(int64_t d, int64_t N, const double* __restrict__ X,
                                                    int64_t ldx, const int64_t* __restrict__ rows,
                                                    double* __restrict__ part) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= d) return;
  const int64_t row = rows ? rows[r] : r;
  const int64_t per = (N + kStatChunks - 1) / kStatChunks;
  const int64_t s0 = blockIdx.y * per, s1 = s0 + per < N ? s0 + per : N;
  double a = 0.0, q = 0.0;
  for (int64_t s = s0; s < s1; ++s) {
    const double v = X[row + s * ldx];
    a += v;
    q += v * v;
  }
  part[(blockIdx.y * d + r) * 2] = a;
  part[(blockIdx.y * d + r) * 2 + 1] = q;
}

__global__ __launch_bounds__(256) void k_stats_fin(int64_t d, int64_t N, const double* __restrict__ part,
                                                   float* __restrict__ mu, float* __restrict__ sd) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= d) return;
  double a = 0.0, q = 0.0;
  for (int c = 0; c < kStatChunks; ++c) {
    a += part[(c * d + r) * 2];
    q += part[(c * d + r) * 2 + 1];
  }
  const double mean = a / (double)N;
  double var = q / (double)N - mean * mean;
  if (!(var > 0.0)) var = 0.0;
  const double s = sqrt(var);
  mu[r] = (float)mean;
  sd[r] = (float)(s > 1e-30 ? s : 1.0);
}

size_t stats_part_size(int64_t d) { return (size_t)kStatChunks * d * 2; }

void launch_stats(hipStream_t s, int64_t d, int64_t N, const double* X, int64_t ldx, const int64_t* rows,
                  double* part, float* mu, float* sd) {
  const unsigned bx = (unsigned)((d + 255) / 256);
  hipLaunchKernelGGL(k_stats_part, dim3(bx, kStatChunks), dim3(256), 0, s, d, N, X, ldx, rows, part);
  hipLaunchKernelGGL(k_stats_fin, dim3(bx), dim3(256), 0, s, d, N, (const double*)part, mu, sd);
}

// Gather a batch: U[r, c] = bf16((X[rows[r] + idx[c] ldx] - mu[r]) / sd[r]) for
// the inputs, and T[i, c] = (Xt[i + idx[c] ldt] - mu_t[i]) / sd_t[i] (FP32)
// for the targets (Xt == null: no targets).  idx == null: sample c0 + c.
__global__ __launch_bounds__(256) void k_gather(int64_t d0, int64_t nb, const double* __restrict__ X,
                                                int64_t ldx, const int64_t* __restrict__ rows,
                                                const float* __restrict__ mu, const float* __restrict__ sd,
                                                const int* __restrict__ idx, int64_t c0,
                                                uint16_t* __restrict__ U, int64_t d3,
                                                const double* __restrict__ Xt, int64_t ldt,
                                                const float* __restrict__ mut, const float* __restrict__ sdt,
                                                float* __restrict__ T) {
  const int64_t c = blockIdx.y;
  const int64_t smp = idx ? (int64_t)idx[c0 + c] : c0 + c;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < d0; r += (int64_t)gridDim.x * 256)
    U[r + c * d0] = f2bf((float)((X[rows[r] + smp * ldx] - (double)mu[r]) / (double)sd[r]));
  if (Xt)
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < d3; i += (int64_t)gridDim.x * 256)
      T[i + c * d3] = (float)((Xt[i + smp * ldt] - (double)mut[i]) / (double)sdt[i]);
}

void launch_gather(hipStream_t s, int64_t d0, int64_t nb, const double* X, int64_t ldx, const int64_t* rows,
                   const float* mu, const float* sd, const int* idx, int64_t c0, uint16_t* U, int64_t d3,
                   const double* Xt, int64_t ldt, const float* mut, const float* sdt, float* T) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3(4, (unsigned)nb), dim3(256), 0, s, d0, nb, X, ldx, rows, mu, sd, idx, c0,
                     U, d3, Xt, ldt, mut, sdt, T);
}

// x0[i, c] = y[i, c] sd_t[i] + mu_t[i] (back from standardised units), FP64 out.
__global__ __launch_bounds__(256) void k_unstd(int64_t d3, int64_t nb, const float* __restrict__ Y,
                                               const float* __restrict__ mut, const float* __restrict__ sdt,
                                               double* __restrict__ X0, int64_t ldx0) {
  const int64_t c = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < d3; i += (int64_t)gridDim.x * 256)
    X0[i + c * ldx0] = (double)Y[i + c * d3] * (double)sdt[i] + (double)mut[i];
}

void launch_unstd(hipStream_t s, int64_t d3, int64_t nb, const float* Y, const float* mut, const float* sdt,
                  double* X0, int64_t ldx0) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_unstd, dim3(4, (unsigned)nb), dim3(256), 0, s, d3, nb, Y, mut, sdt, X0, ldx0);
}

}  // namespace ils
