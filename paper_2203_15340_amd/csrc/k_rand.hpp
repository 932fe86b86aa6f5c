// k_rand.hpp -- launchers of the randomized inner-loop kernels (k_rand.hip).
#pragma once
#include "ils_common.hpp"

namespace ils {

constexpr int64_t kScdMaxN = 4096;  // largest n for SP-SCD with random subsets (LDS keys)

void launch_prefix(hipStream_t s, int64_t n, const double* w, int64_t stride, double* prefix);
void launch_rk_draw(hipStream_t s, uint64_t seed, uint64_t outer, int64_t t0, int64_t count,
                    const double* prefix, int64_t n, int* j1, int* j2);
void launch_scd_draw(hipStream_t s, uint64_t seed, uint64_t outer, int64_t t0, int64_t count, int64_t n,
                     int64_t alpha_opt, int norm_mode, const double* prefix, int* alpha, int* jout,
                     uint32_t* mask, int64_t mask_words);
void launch_rk_inner(hipStream_t st, const double* A1, int64_t lda, int64_t p, const double* tgt,
                     const double* cn, const int* j1, const int* j2, int64_t count, double* w, double* s,
                     double* z, const int* inner_done, const int* outer_done);
void launch_rk_check(hipStream_t st, const double* A1, int64_t lda, int64_t p, int64_t n, const double* w,
                     const double* s, double* v, const double* tgt, double* res2, double itol2,
                     const double* tn2, int* inner_done, unsigned* arrive, const int* skip);
void launch_rk_inner_f32(hipStream_t st, const float* A1, int64_t lda, int64_t p, const double* tgt,
                         const double* cn, const int* j1, const int* j2, int64_t count, float* w, float* s,
                         double* z, const int* inner_done, const int* outer_done);
void launch_rk_check_f32(hipStream_t st, const double* A1, int64_t lda, int64_t p, int64_t n, const float* w,
                         const float* s, double* v, const double* tgt, double* res2, double itol2,
                         const double* tn2, int* inner_done, unsigned* arrive, const int* skip);
void launch_to_f32(hipStream_t s, int64_t p, int64_t n, const double* A, int64_t lda, float* Af);
// SP-RK-RGS inner steps in blocks spread over the GPU (k_rkblock.hip);
// scratch: rk_block_scratch(p) doubles; arrive: a zero last-block counter
// (left zero).
int64_t rk_block_steps();
int64_t rk_block_slice_rows(int64_t p);
size_t rk_block_scratch(int64_t p);
void launch_rk_blocks(hipStream_t st, const double* A1, int64_t lda, int64_t p, const double* tgt, const double* cn,
                      const int* j1, const int* j2, int64_t count, double* w, double* s, double* z, double* scratch,
                      unsigned* arrive, const int* inner_done, const int* outer_done);
void launch_rk_blocks_f32(hipStream_t st, const float* A1, int64_t lda, int64_t p, const double* tgt,
                          const double* cn, const int* j1, const int* j2, int64_t count, float* w, float* s,
                          double* z, double* scratch, unsigned* arrive, const int* inner_done,
                          const int* outer_done);
// SP-RK-RGS blocks for up to kMR right-hand sides sharing one index stream
// (k_rkmulti.hip).  W, S: p x R (ldw), Z, tgt: n x R; frozen: R flags (a
// frozen right-hand side takes zero coefficients); scratch:
// rk_multi_scratch(p) doubles; arrive: a zero last-block counter.
constexpr int kMR = 16;
size_t rk_multi_scratch(int64_t p);
void launch_rk_multi_blocks(hipStream_t st, const double* A1, int64_t lda, int64_t p, int R, const double* tgt,
                            int64_t ldt, const double* cn, const int* j1, const int* j2, int64_t count,
                            double* W, double* S, int64_t ldw, double* Z, int64_t ldz, const int* frozen,
                            double* scratch, unsigned* arrive);
// Inner stop test of every right-hand side of a group: V (p x R) and AtV
// (n x R) are scratch; sets frozen[r] when ||tgt_r - A1^T (w_r - s_r)||^2 <=
// itol2 tn2[r].
void launch_rkm_check(hipStream_t st, const double* A1, int64_t lda, int64_t p, int64_t n, int R, const double* W,
                      const double* S, int64_t ldw, double* V, double* AtV, const double* tgt, int64_t ldt,
                      const double* tn2, double itol2, int* frozen);
void launch_scd_inner(hipStream_t st, const double* G1, int64_t ldg, int64_t n, double* r, double* beta,
                      const uint32_t* mask, int64_t mask_words, const int* jpre, int norm_mode,
                      int64_t count, int check, double itol2, const double* tn2, int* inner_done,
                      int64_t* steps_done, const int* outer_done);
// The same steps with G1 and r in FP32 (mixed precision; beta stays FP64).
void launch_scd_inner_f32(hipStream_t st, const float* G1, int64_t ldg, int64_t n, float* r, double* beta,
                          const uint32_t* mask, int64_t mask_words, const int* jpre, int norm_mode,
                          int64_t count, int check, double itol2, const double* tn2, int* inner_done,
                          int64_t* steps_done, const int* outer_done);
void launch_symv_add(hipStream_t s, int64_t n, const double* G, int64_t ldg, const double* x,
                     const double* g, double* y, const int* skip);
void launch_outer_test(hipStream_t s, int64_t n, const double* xk, const double* x_ref, const double* rk,
                       int stop_rule, double tol, int64_t k, int64_t max_outer, LoopState* st);
void launch_outer_update(hipStream_t s, int64_t n, const double* xk, const double* z, int correction,
                         double* xn, int64_t k, LoopState* st);
void launch_diag(hipStream_t s, int64_t n, const double* G, int64_t ldg, double* d);
void launch_zero_col_check(hipStream_t s, int64_t n, const double* c, int* bits);

}  // namespace ils
