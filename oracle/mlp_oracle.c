/* mlp_oracle.c -- plain FP64 reference of the warm-start network.
 *
 * TEST INFRASTRUCTURE ONLY (see ils_oracle.h).  Shares no code with the GPU
 * library.
 *
 * The network maps a (standardised) row sample of b to a (standardised)
 * estimate of x, used as the initial value x0 of the SP iteration; SP
 * converges from any x0 (Thm. 2.1), so the network only changes the number of
 * outer steps.  It is a three-layer perceptron
 *     h1 = relu(W1 u + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3
 * with W_l of size d_l x d_{l-1} stored row-major (W[o * d_{l-1} + i]).  The
 * parameter vector theta is [W1, b1, W2, b2, W3, b3] in that order.
 * Loss over a batch of B samples: L = (1 / (B d3)) sum (y - t)^2.
 * Inputs U (d0 x B) and targets T (d3 x B) are column-major, one sample per
 * column.
 *
 * Adam (Kingma & Ba, ICLR 2015, Algorithm 1): m <- b1 m + (1-b1) g,
 * v <- b2 v + (1-b2) g^2, w <- w - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "ils_oracle.h"

int64_t ora_mlp_nparams(const int64_t d[4]) {
  return d[1] * d[0] + d[1] + d[2] * d[1] + d[2] + d[3] * d[2] + d[3];
}

/* offsets of W_l and b_l inside theta */
static void layout(const int64_t d[4], int64_t offW[3], int64_t offb[3]) {
  int64_t o = 0;
  for (int l = 0; l < 3; ++l) {
    offW[l] = o;
    o += d[l + 1] * d[l];
    offb[l] = o;
    o += d[l + 1];
  }
}

/* out (dout x B) = W in + b, optionally through relu */
static void dense_layer(int64_t din, int64_t dout, const double* W, const double* bias, int64_t B,
                        const double* in, double* out, int relu) {
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < B; ++s) {
    for (int64_t o = 0; o < dout; ++o) {
      double acc = bias[o];
      for (int64_t i = 0; i < din; ++i) acc += W[o * din + i] * in[s * din + i];
      out[s * dout + o] = (relu && acc < 0.0) ? 0.0 : acc;
    }
  }
}

void ora_mlp_forward(const int64_t d[4], const double* theta, int64_t B, const double* U,
                     double* Y, double* H1, double* H2) {
  int64_t oW[3], ob[3];
  layout(d, oW, ob);
  double* h1 = H1 ? H1 : (double*)malloc(sizeof(double) * (size_t)(d[1] * B));
  double* h2 = H2 ? H2 : (double*)malloc(sizeof(double) * (size_t)(d[2] * B));
  dense_layer(d[0], d[1], theta + oW[0], theta + ob[0], B, U, h1, 1);
  dense_layer(d[1], d[2], theta + oW[1], theta + ob[1], B, h1, h2, 1);
  dense_layer(d[2], d[3], theta + oW[2], theta + ob[2], B, h2, Y, 0);
  if (!H1) free(h1);
  if (!H2) free(h2);
}

double ora_mlp_loss(const int64_t d[4], const double* theta, int64_t B, const double* U,
                    const double* T) {
  double* Y = (double*)malloc(sizeof(double) * (size_t)(d[3] * B));
  ora_mlp_forward(d, theta, B, U, Y, NULL, NULL);
  double s = 0.0;
  for (int64_t k = 0; k < d[3] * B; ++k) s += (Y[k] - T[k]) * (Y[k] - T[k]);
  free(Y);
  return s / (double)(B * d[3]);
}

/* Backward pass by the chain rule, layer by layer from the output:
 * dY = 2 (y - t) / (B d3); for a layer out = f(W in + b):
 *   dZ = dOut * f'(Z) (f' = 1[out > 0] for relu), dW = dZ in^T, db = sum_s dZ,
 *   dIn = W^T dZ. */
double ora_mlp_grad(const int64_t d[4], const double* theta, int64_t B, const double* U,
                    const double* T, double* grad) {
  int64_t oW[3], ob[3];
  layout(d, oW, ob);
  double* h1 = (double*)malloc(sizeof(double) * (size_t)(d[1] * B));
  double* h2 = (double*)malloc(sizeof(double) * (size_t)(d[2] * B));
  double* Y = (double*)malloc(sizeof(double) * (size_t)(d[3] * B));
  ora_mlp_forward(d, theta, B, U, Y, h1, h2);
  double loss = 0.0;
  double* dz = (double*)malloc(sizeof(double) * (size_t)(d[3] * B));
  for (int64_t k = 0; k < d[3] * B; ++k) {
    loss += (Y[k] - T[k]) * (Y[k] - T[k]);
    dz[k] = 2.0 * (Y[k] - T[k]) / (double)(B * d[3]);
  }
  loss /= (double)(B * d[3]);
  const double* ins[3] = {U, h1, h2};
  for (int l = 2; l >= 0; --l) {
    const int64_t din = d[l], dout = d[l + 1];
    const double* in = ins[l];
    const double* W = theta + oW[l];
    double* gW = grad + oW[l];
    double* gb = grad + ob[l];
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < dout; ++o) {
      double sb = 0.0;
      for (int64_t s = 0; s < B; ++s) sb += dz[s * dout + o];
      gb[o] = sb;
      for (int64_t i = 0; i < din; ++i) {
        double sw = 0.0;
        for (int64_t s = 0; s < B; ++s) sw += dz[s * dout + o] * in[s * din + i];
        gW[o * din + i] = sw;
      }
    }
    if (l == 0) break;
    /* gradient with respect to the layer input, through the previous relu */
    double* dprev = (double*)malloc(sizeof(double) * (size_t)(din * B));
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < B; ++s) {
      for (int64_t i = 0; i < din; ++i) {
        double acc = 0.0;
        for (int64_t o = 0; o < dout; ++o) acc += W[o * din + i] * dz[s * dout + o];
        dprev[s * din + i] = in[s * din + i] > 0.0 ? acc : 0.0;
      }
    }
    free(dz);
    dz = dprev;
  }
  free(dz);
  free(Y);
  free(h2);
  free(h1);
  return loss;
}

void ora_adam_step(int64_t len, double* w, double* m, double* v, const double* g, int64_t t,
                   double lr, double beta1, double beta2, double eps) {
  const double c1 = 1.0 - pow(beta1, (double)t);
  const double c2 = 1.0 - pow(beta2, (double)t);
  for (int64_t k = 0; k < len; ++k) {
    m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
    v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
    w[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
  }
}

/* Round to the nearest bfloat16 (8 significand bits), ties to even: the
 * value the GPU sees for a weight or input stored in that format. */
double ora_bf16_round(double x) {
  if (!isfinite(x) || x == 0.0) return x;
  int e;
  double f = frexp(x, &e);        /* x = f 2^e, 0.5 <= |f| < 1 */
  double s = ldexp(f, 8);         /* 8 significant bits left of the point */
  double r = nearbyint(s);        /* default rounding mode: ties to even */
  return ldexp(r, e - 8);
}
