// ils_ws_api.hip -- the learned warm start: a three-layer BF16 perceptron
// that maps a row sample of b to an initial value x0 for SP (Alg. 1
// converges from any x0, Thm. 2.1, so the network changes only the number
// of outer steps).  Training and inference run on the kernels of k_mlp.hip;
// the host side here owns the buffers, the epoch loop, the sample shuffle
// and the file format.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ils_common.hpp"
#include "ils_runtime.hpp"
#include "k_mlp.hpp"

using namespace ils;

#define HIPCHK(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return ILS_ERR_HIP; \
  } while (0)

struct ils_ws {
  ils_handle* h = nullptr;
  int64_t m = 0, n = 0, d[4] = {};
  int64_t np = 0, offW[3] = {}, offb[3] = {};
  uint64_t seed = 0;
  int64_t t = 0;  // Adam steps taken
  std::vector<int64_t> rows_host;
  int64_t* rows = nullptr;
  int64_t* seg = nullptr;
  float *theta = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;
  uint16_t* wb = nullptr;
  float *mu_in = nullptr, *sd_in = nullptr, *mu_out = nullptr, *sd_out = nullptr;
  // per-batch buffers, sized for `cap` samples
  int64_t cap = 0;
  uint16_t *U = nullptr, *H1 = nullptr, *H2 = nullptr, *dZb = nullptr;
  float *Y = nullptr, *T = nullptr, *dZf = nullptr;
  double* loss_rows = nullptr;
  double* losses = nullptr;
  int64_t losses_cap = 0;
  int* idx = nullptr;
  int* idx_host = nullptr;  // pinned
  int64_t idx_cap = 0;
  double* stat_part = nullptr;
  int64_t stat_cap = 0;
  ~ils_ws();
};

ils_ws::~ils_ws() {
  void* dev[] = {rows, seg, theta, m1, m2, grad, wb, mu_in, sd_in, mu_out, sd_out, U, H1, H2, dZb, Y, T,
                 dZf, loss_rows, losses, idx, stat_part};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (idx_host) (void)hipHostFree(idx_host);
}

template <typename T>
static int dalloc(T** p, size_t count) {
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, sizeof(T) * count) == hipSuccess ? ILS_OK : ILS_ERR_ALLOC;
}

static int ensure_cap(ils_ws* w, int64_t nb) {
  if (nb <= w->cap) return ILS_OK;
  const int64_t c = std::max<int64_t>(nb, 256);
  const int64_t dh = std::max(w->d[1], w->d[2]);
  const int64_t dz = std::max(dh, w->d[3]);
  int st;
  if ((st = dalloc(&w->U, w->d[0] * c)) || (st = dalloc(&w->H1, w->d[1] * c)) ||
      (st = dalloc(&w->H2, w->d[2] * c)) || (st = dalloc(&w->dZb, dz * c)) ||
      (st = dalloc(&w->Y, w->d[3] * c)) || (st = dalloc(&w->T, w->d[3] * c)) || (st = dalloc(&w->dZf, dh * c)))
    return st;
  w->cap = c;
  return ILS_OK;
}

// ------------------------------------------------------------------ passes
// Forward over nb samples already in w->U: H1, H2 (bf16) and Y (FP32).
static void forward(ils_ws* w, hipStream_t s, int64_t nb) {
  const int64_t* d = w->d;
  MlpGemmArgs g = {};
  g.N = nb;
  // h1 = relu(W1 u + b1)
  g.M = d[1]; g.K = d[0]; g.A = w->wb + w->offW[0]; g.lda = d[0]; g.B = w->U; g.ldb = d[0];
  g.bias = w->theta + w->offb[0]; g.Cb = w->H1; g.ldc = d[1];
  launch_mlp_gemm(s, 1, 0, kEpiBiasReluBf16, g);
  // h2 = relu(W2 h1 + b2)
  g.M = d[2]; g.K = d[1]; g.A = w->wb + w->offW[1]; g.lda = d[1]; g.B = w->H1; g.ldb = d[1];
  g.bias = w->theta + w->offb[1]; g.Cb = w->H2; g.ldc = d[2];
  launch_mlp_gemm(s, 1, 0, kEpiBiasReluBf16, g);
  // y = W3 h2 + b3
  g.M = d[3]; g.K = d[2]; g.A = w->wb + w->offW[2]; g.lda = d[2]; g.B = w->H2; g.ldb = d[2];
  g.bias = w->theta + w->offb[2]; g.Cb = nullptr; g.Cf = w->Y; g.ldc = d[3];
  launch_mlp_gemm(s, 1, 0, kEpiBiasF32, g);
}

// Backward for the MSE loss against w->T: gradient into w->grad, loss into *loss.
static void backward(ils_ws* w, hipStream_t s, int64_t nb, double* loss) {
  const int64_t* d = w->d;
  launch_mlp_outgrad(s, d[3], nb, w->Y, w->T, w->dZb, w->grad + w->offb[2], w->loss_rows, loss);
  for (int l = 2; l >= 0; --l) {
    const int64_t dout = d[l + 1], din = d[l];
    const uint16_t* in = l == 0 ? w->U : (l == 1 ? w->H1 : w->H2);
    // dW_l = dZ_l in^T, stored row-major into theta's layout
    MlpGemmArgs g = {};
    g.M = dout; g.N = din; g.K = nb;
    g.A = w->dZb; g.lda = dout; g.B = in; g.ldb = din;
    g.Cf = w->grad + w->offW[l]; g.csi = din; g.csj = 1;
    launch_mlp_gemm(s, 0, 1, kEpiStoreF32, g);
    if (l == 0) break;
    // dZ_{l-1} = (W_l^T dZ_l) * 1[h_{l-1} > 0]
    MlpGemmArgs b = {};
    b.M = din; b.N = nb; b.K = dout;
    b.A = w->wb + w->offW[l]; b.lda = din; b.B = w->dZb; b.ldb = dout;
    b.mask = in; b.ldmask = din; b.Cf = w->dZf; b.ldc = din;
    launch_mlp_gemm(s, 0, 0, kEpiMaskF32, b);
    launch_mlp_rowsum(s, din, nb, w->dZf, w->dZb, w->grad + w->offb[l - 1]);
  }
}

static void adam(ils_ws* w, hipStream_t s, double lr) {
  ++w->t;
  const double b1 = 0.9, b2 = 0.999;
  AdamArgs a;
  a.lr = (float)lr;
  a.b1 = (float)b1;
  a.b2 = (float)b2;
  a.omb1 = (float)(1.0 - b1);
  a.omb2 = (float)(1.0 - b2);
  a.eps = 1e-8f;
  a.c1 = (float)(1.0 - pow(b1, (double)w->t));
  a.c2 = (float)(1.0 - pow(b2, (double)w->t));
  launch_adam(s, w->np, w->theta, w->m1, w->m2, w->grad, w->wb, a);
}

// ------------------------------------------------------------------ C ABI
extern "C" int ils_ws_create(ils_handle* h, int64_t m, int64_t n, int64_t d_in, const int64_t* in_rows,
                             int64_t hidden, uint64_t seed, ils_ws** out) {
  if (!h || !out || !in_rows || m < 1 || n < 1 || d_in < 1 || hidden < 1) return ILS_ERR_ARG;
  if (d_in > m || n > (1 << 20) || hidden > (1 << 16) || d_in > (1 << 24)) return ILS_ERR_ARG;
  for (int64_t r = 0; r < d_in; ++r)
    if (in_rows[r] < 0 || in_rows[r] >= m) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(h->device));
  ils_ws* w = new ils_ws();
  w->h = h;
  w->m = m;
  w->n = n;
  w->d[0] = d_in;
  w->d[1] = hidden;
  w->d[2] = hidden;
  w->d[3] = n;
  w->seed = seed;
  int64_t o = 0;
  for (int l = 0; l < 3; ++l) {
    w->offW[l] = o;
    o += w->d[l + 1] * w->d[l];
    w->offb[l] = o;
    o += w->d[l + 1];
  }
  w->np = o;
  w->rows_host.assign(in_rows, in_rows + d_in);
  int64_t seg[10] = {w->offW[0], w->offb[0], w->offW[1], w->offb[1], w->offW[2], w->offb[2], w->np,
                     w->d[0], w->d[1], w->d[2]};
  hipStream_t s = h->stream;
  int st;
  if ((st = dalloc(&w->rows, d_in)) || (st = dalloc(&w->seg, 10)) || (st = dalloc(&w->theta, w->np)) ||
      (st = dalloc(&w->m1, w->np)) || (st = dalloc(&w->m2, w->np)) || (st = dalloc(&w->grad, w->np)) ||
      (st = dalloc(&w->wb, w->np)) || (st = dalloc(&w->mu_in, d_in)) || (st = dalloc(&w->sd_in, d_in)) ||
      (st = dalloc(&w->mu_out, n)) || (st = dalloc(&w->sd_out, n)) || (st = dalloc(&w->loss_rows, n))) {
    delete w;
    return st;
  }
  if (hipMemcpyAsync(w->rows, in_rows, sizeof(int64_t) * d_in, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(w->seg, seg, sizeof(seg), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(w->m1, 0, sizeof(float) * w->np, s) != hipSuccess ||
      hipMemsetAsync(w->m2, 0, sizeof(float) * w->np, s) != hipSuccess ||
      hipMemsetAsync(w->mu_in, 0, sizeof(float) * d_in, s) != hipSuccess ||
      hipMemsetAsync(w->mu_out, 0, sizeof(float) * n, s) != hipSuccess) {
    delete w;
    return ILS_ERR_HIP;
  }
  std::vector<float> ones(std::max(d_in, n), 1.0f);
  launch_mlp_init(s, w->np, w->seg, w->theta, seed);
  launch_f2bf(s, w->np, w->theta, w->wb);
  if (hipMemcpyAsync(w->sd_in, ones.data(), sizeof(float) * d_in, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(w->sd_out, ones.data(), sizeof(float) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    delete w;
    return ILS_ERR_HIP;
  }
  *out = w;
  return ILS_OK;
}

extern "C" int ils_ws_destroy(ils_ws* w) {
  if (!w) return ILS_ERR_ARG;
  (void)hipSetDevice(w->h->device);
  (void)hipStreamSynchronize(w->h->stream);
  delete w;
  return ILS_OK;
}

extern "C" int ils_ws_nparams(const ils_ws* w, int64_t* np) {
  if (!w || !np) return ILS_ERR_ARG;
  *np = w->np;
  return ILS_OK;
}

extern "C" int ils_ws_get_params(ils_ws* w, float* theta) {
  if (!w || !theta) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(w->h->device));
  HIPCHK(hipMemcpyAsync(theta, w->theta, sizeof(float) * w->np, hipMemcpyDeviceToDevice, w->h->stream));
  HIPCHK(hipStreamSynchronize(w->h->stream));
  return ILS_OK;
}

extern "C" int ils_ws_set_params(ils_ws* w, const float* theta) {
  if (!w || !theta) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(w->h->device));
  hipStream_t s = w->h->stream;
  HIPCHK(hipMemcpyAsync(w->theta, theta, sizeof(float) * w->np, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemsetAsync(w->m1, 0, sizeof(float) * w->np, s));
  HIPCHK(hipMemsetAsync(w->m2, 0, sizeof(float) * w->np, s));
  launch_f2bf(s, w->np, w->theta, w->wb);
  w->t = 0;
  HIPCHK(hipStreamSynchronize(s));
  return ILS_OK;
}

// Standardised inputs (FP32, rounded to bf16 here) -> network output / gradient.
static int load_inputs(ils_ws* w, int64_t N, const float* U, const float* T) {
  int st = ensure_cap(w, N);
  if (st) return st;
  hipStream_t s = w->h->stream;
  launch_f2bf(s, w->d[0] * N, U, w->U);
  if (T) HIPCHK(hipMemcpyAsync(w->T, T, sizeof(float) * w->d[3] * N, hipMemcpyDeviceToDevice, s));
  return ILS_OK;
}

extern "C" int ils_ws_forward(ils_ws* w, int64_t N, const float* U, float* Y) {
  if (!w || !U || !Y || N < 1) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(w->h->device));
  int st = load_inputs(w, N, U, nullptr);
  if (st) return st;
  hipStream_t s = w->h->stream;
  forward(w, s, N);
  HIPCHK(hipMemcpyAsync(Y, w->Y, sizeof(float) * w->d[3] * N, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return ILS_OK;
}

extern "C" int ils_ws_grad(ils_ws* w, int64_t N, const float* U, const float* T, float* grad, double* loss) {
  if (!w || !U || !T || !grad || N < 1) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(w->h->device));
  int st = load_inputs(w, N, U, T);
  if (st) return st;
  if (w->losses_cap < 1 && (st = dalloc(&w->losses, 1024))) return st;
  w->losses_cap = std::max<int64_t>(w->losses_cap, 1024);
  hipStream_t s = w->h->stream;
  forward(w, s, N);
  backward(w, s, N, w->losses);
  HIPCHK(hipMemcpyAsync(grad, w->grad, sizeof(float) * w->np, hipMemcpyDeviceToDevice, s));
  double l = 0.0;
  HIPCHK(hipMemcpyAsync(&l, w->losses, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  if (loss) *loss = l;
  return ILS_OK;
}

extern "C" int ils_ws_adam(ils_ws* w, const float* grad, double lr) {
  if (!w || !grad || !(lr > 0.0)) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(w->h->device));
  hipStream_t s = w->h->stream;
  HIPCHK(hipMemcpyAsync(w->grad, grad, sizeof(float) * w->np, hipMemcpyDeviceToDevice, s));
  adam(w, s, lr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return ILS_OK;
}

// SplitMix64 stream for the epoch shuffle (Fisher-Yates).
static uint64_t sm64(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

extern "C" int ils_ws_train(ils_ws* w, int64_t N, const double* B, int64_t ldb, const double* X, int64_t ldx,
                            int32_t epochs, int64_t batch, double lr, double* final_loss) {
  if (!w || !B || !X || N < 1 || N > ((int64_t)1 << 31) - 1 || ldb < w->m || ldx < w->n || epochs < 0 ||
      batch < 1 || !(lr > 0.0))
    return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(w->h->device));
  hipStream_t s = w->h->stream;
  int st;
  if ((st = ensure_cap(w, batch))) return st;
  const int64_t nbatches = (N + batch - 1) / batch;
  if (nbatches > w->losses_cap) {
    if ((st = dalloc(&w->losses, std::max<int64_t>(nbatches, 1024)))) return st;
    w->losses_cap = std::max<int64_t>(nbatches, 1024);
  }
  if (N > w->idx_cap) {
    if ((st = dalloc(&w->idx, N))) return st;
    if (w->idx_host) (void)hipHostFree(w->idx_host);
    w->idx_host = nullptr;
    HIPCHK(hipHostMalloc((void**)&w->idx_host, sizeof(int) * N, hipHostMallocDefault));
    w->idx_cap = N;
  }
  const int64_t dstat = std::max(w->d[0], w->d[3]);
  if ((int64_t)stats_part_size(dstat) > w->stat_cap) {
    if ((st = dalloc(&w->stat_part, stats_part_size(dstat)))) return st;
    w->stat_cap = (int64_t)stats_part_size(dstat);
  }
  // standardisation of this training set (inputs: the sampled rows of b)
  launch_stats(s, w->d[0], N, B, ldb, w->rows, w->stat_part, w->mu_in, w->sd_in);
  launch_stats(s, w->d[3], N, X, ldx, nullptr, w->stat_part, w->mu_out, w->sd_out);
  HIPCHK(hipGetLastError());
  std::vector<double> hl(nbatches);
  double last = NAN;
  for (int32_t e = 0; e < epochs; ++e) {
    uint64_t state = w->seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(w->t + 1));
    for (int64_t i = 0; i < N; ++i) w->idx_host[i] = (int)i;
    for (int64_t i = N - 1; i > 0; --i) {
      const int64_t j = (int64_t)(((unsigned __int128)sm64(state) * (uint64_t)(i + 1)) >> 64);
      std::swap(w->idx_host[i], w->idx_host[j]);
    }
    HIPCHK(hipMemcpyAsync(w->idx, w->idx_host, sizeof(int) * N, hipMemcpyHostToDevice, s));
    for (int64_t bi = 0; bi < nbatches; ++bi) {
      const int64_t c0 = bi * batch, nb = std::min(batch, N - c0);
      launch_gather(s, w->d[0], nb, B, ldb, w->rows, w->mu_in, w->sd_in, w->idx, c0, w->U, w->d[3], X, ldx,
                    w->mu_out, w->sd_out, w->T);
      forward(w, s, nb);
      backward(w, s, nb, w->losses + bi);
      adam(w, s, lr);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hl.data(), w->losses, sizeof(double) * nbatches, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double sum = 0.0, cnt = 0.0;
    for (int64_t bi = 0; bi < nbatches; ++bi) {
      const double nb = (double)std::min(batch, N - bi * batch);
      sum += hl[bi] * nb;
      cnt += nb;
    }
    last = sum / cnt;
    if (!isfinite(last)) {
      if (final_loss) *final_loss = last;
      return ILS_ERR_NONFINITE;
    }
  }
  if (final_loss) *final_loss = last;
  return ILS_OK;
}

extern "C" int ils_ws_infer(ils_ws* w, int64_t N, const double* B, int64_t ldb, double* X0, int64_t ldx0) {
  if (!w || !B || !X0 || N < 1 || ldb < w->m || ldx0 < w->n) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(w->h->device));
  hipStream_t s = w->h->stream;
  const int64_t chunk = 4096;
  int st = ensure_cap(w, std::min(N, chunk));
  if (st) return st;
  for (int64_t c0 = 0; c0 < N; c0 += w->cap) {
    const int64_t nb = std::min(w->cap, N - c0);
    launch_gather(s, w->d[0], nb, B, ldb, w->rows, w->mu_in, w->sd_in, nullptr, c0, w->U, w->d[3], nullptr,
                  0, nullptr, nullptr, nullptr);
    forward(w, s, nb);
    launch_unstd(s, w->d[3], nb, w->Y, w->mu_out, w->sd_out, X0 + c0 * ldx0, ldx0);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return ILS_OK;
}

// ------------------------------------------------------------------ files
// Layout: 8-byte magic, int64 m, n, d[4], t, uint64 seed, int64 rows[d0],
// float mu_in[d0], sd_in[d0], mu_out[n], sd_out[n], theta[np], m1[np], m2[np].
static const char kMagic[8] = {'I', 'L', 'S', 'W', 'S', 0, 0, 1};

extern "C" int ils_ws_save(ils_ws* w, const char* path) {
  if (!w || !path) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(w->h->device));
  hipStream_t s = w->h->stream;
  const int64_t d0 = w->d[0], n = w->n, np = w->np;
  std::vector<float> f(2 * d0 + 2 * n + 3 * np);
  float* p = f.data();
  HIPCHK(hipMemcpyAsync(p, w->mu_in, sizeof(float) * d0, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(p + d0, w->sd_in, sizeof(float) * d0, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(p + 2 * d0, w->mu_out, sizeof(float) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(p + 2 * d0 + n, w->sd_out, sizeof(float) * n, hipMemcpyDeviceToHost, s));
  float* q = p + 2 * d0 + 2 * n;
  HIPCHK(hipMemcpyAsync(q, w->theta, sizeof(float) * np, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(q + np, w->m1, sizeof(float) * np, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(q + 2 * np, w->m2, sizeof(float) * np, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  FILE* fp = fopen(path, "wb");
  if (!fp) return ILS_ERR_ARG;
  int64_t hdr[8] = {w->m, w->n, w->d[0], w->d[1], w->d[2], w->d[3], w->t, (int64_t)w->seed};
  bool ok = fwrite(kMagic, 1, 8, fp) == 8 && fwrite(hdr, sizeof(hdr), 1, fp) == 1 &&
            fwrite(w->rows_host.data(), sizeof(int64_t), d0, fp) == (size_t)d0 &&
            fwrite(f.data(), sizeof(float), f.size(), fp) == f.size();
  ok = (fclose(fp) == 0) && ok;
  return ok ? ILS_OK : ILS_ERR_ARG;
}

extern "C" int ils_ws_load(ils_ws* w, const char* path) {
  if (!w || !path) return ILS_ERR_ARG;
  FILE* fp = fopen(path, "rb");
  if (!fp) return ILS_ERR_ARG;
  char magic[8];
  int64_t hdr[8];
  const int64_t d0 = w->d[0], n = w->n, np = w->np;
  std::vector<int64_t> rows(d0);
  std::vector<float> f(2 * d0 + 2 * n + 3 * np);
  bool ok = fread(magic, 1, 8, fp) == 8 && memcmp(magic, kMagic, 8) == 0 && fread(hdr, sizeof(hdr), 1, fp) == 1 &&
            hdr[0] == w->m && hdr[1] == w->n && hdr[2] == w->d[0] && hdr[3] == w->d[1] && hdr[4] == w->d[2] &&
            hdr[5] == w->d[3] && fread(rows.data(), sizeof(int64_t), d0, fp) == (size_t)d0 &&
            fread(f.data(), sizeof(float), f.size(), fp) == f.size();
  fclose(fp);
  if (!ok) return ILS_ERR_ARG;
  for (int64_t r = 0; r < d0; ++r)
    if (rows[r] < 0 || rows[r] >= w->m) return ILS_ERR_ARG;
  HIPCHK(hipSetDevice(w->h->device));
  hipStream_t s = w->h->stream;
  const float* p = f.data();
  const float* q = p + 2 * d0 + 2 * n;
  HIPCHK(hipMemcpyAsync(w->rows, rows.data(), sizeof(int64_t) * d0, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w->mu_in, p, sizeof(float) * d0, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w->sd_in, p + d0, sizeof(float) * d0, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w->mu_out, p + 2 * d0, sizeof(float) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w->sd_out, p + 2 * d0 + n, sizeof(float) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w->theta, q, sizeof(float) * np, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w->m1, q + np, sizeof(float) * np, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w->m2, q + 2 * np, sizeof(float) * np, hipMemcpyHostToDevice, s));
  launch_f2bf(s, np, w->theta, w->wb);
  HIPCHK(hipStreamSynchronize(s));
  w->rows_host = rows;
  w->t = hdr[6];
  w->seed = (uint64_t)hdr[7];
  return ILS_OK;
}
