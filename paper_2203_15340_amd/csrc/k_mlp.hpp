// k_mlp.hpp -- launchers of the warm-start network kernels (k_mlp.hip).
#pragma once
#include "ils_common.hpp"

namespace ils {

enum : int {
  kEpiBiasReluBf16 = 0,  // Cb = bf16(relu(acc + bias[i]))
  kEpiBiasF32 = 1,       // Cf = acc + bias[i]
  kEpiMaskF32 = 2,       // Cf = mask[i, j] != 0 ? acc : 0
  kEpiStoreF32 = 3,      // Cf[i csi + j csj] = acc
};

struct MlpGemmArgs {
  int64_t M, N, K;
  const uint16_t* A;
  int64_t lda;
  const uint16_t* B;
  int64_t ldb;
  const float* bias;
  const uint16_t* mask;
  int64_t ldmask;
  uint16_t* Cb;
  float* Cf;
  int64_t ldc;
  int64_t csi, csj;
};

void launch_mlp_gemm(hipStream_t s, int ta, int tb, int epi, const MlpGemmArgs& g);
void launch_f2bf(hipStream_t s, int64_t n, const float* x, uint16_t* y);
void launch_mlp_outgrad(hipStream_t s, int64_t d3, int64_t N, const float* Y, const float* T, uint16_t* dYb,
                        float* db, double* loss_rows, double* loss);
void launch_mlp_rowsum(hipStream_t s, int64_t d, int64_t N, const float* dZ, uint16_t* dZb, float* db);
struct AdamArgs {
  float lr, b1, b2, omb1, omb2, eps, c1, c2;
};
void launch_adam(hipStream_t s, int64_t n, float* w, float* m, float* v, const float* g, uint16_t* wb,
                 const AdamArgs& a);
void launch_mlp_init(hipStream_t s, int64_t n, const int64_t* seg, float* w, uint64_t seed);
size_t stats_part_size(int64_t d);
void launch_stats(hipStream_t s, int64_t d, int64_t N, const double* X, int64_t ldx, const int64_t* rows,
                  double* part, float* mu, float* sd);
void launch_gather(hipStream_t s, int64_t d0, int64_t nb, const double* X, int64_t ldx, const int64_t* rows,
                   const float* mu, const float* sd, const int* idx, int64_t c0, uint16_t* U, int64_t d3,
                   const double* Xt, int64_t ldt, const float* mut, const float* sdt, float* T);
void launch_unstd(hipStream_t s, int64_t d3, int64_t nb, const float* Y, const float* mut, const float* sdt,
                  double* X0, int64_t ldx0);

}  // namespace ils
