/*
 * Oracle (test infrastructure only): the per-node closure network and its
 * training step, in plain FP64.
 *
 * The paper does not define a learned closure; this is the network the GPU
 * path implements for it, written out as its definition:
 *
 *   z1 = W1 x + b1,  h1 = g(z1)          (4 -> 64)
 *   z2 = W2 h1 + b2, h2 = g(z2)          (64 -> 64)
 *   z3 = W3 h2 + b3, h3 = g(z3)          (64 -> 64)
 *   y  = W4 h3 + b4                      (64 -> 2)
 *
 * with g the rectifier g(z) = max(z, 0) (derivative 1 for z > 0, else 0).
 * Parameters are packed in one array, weights row-major [out][in]:
 *   W1[64][4] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[2][64] b4[2]
 * (8770 values).  The loss of a batch is L = 1/(2n) sum_s sum_o (y_so - t_so)^2
 * and its gradient is taken by the chain rule, layer by layer backwards.
 * Adam follows Kingma and Ba (bias-corrected first and second moments).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define H OR_MLP_HIDDEN

/* offsets of the parameter blocks */
enum {
  OFF_W1 = 0,
  OFF_B1 = OFF_W1 + H * OR_MLP_IN,
  OFF_W2 = OFF_B1 + H,
  OFF_B2 = OFF_W2 + H * H,
  OFF_W3 = OFF_B2 + H,
  OFF_B3 = OFF_W3 + H * H,
  OFF_W4 = OFF_B3 + H,
  OFF_B4 = OFF_W4 + OR_MLP_OUT * H,
  OFF_END = OFF_B4 + OR_MLP_OUT
};

double or_relu(double z) { return z > 0.0 ? z : 0.0; }

double or_relu_d(double z) { return z > 0.0 ? 1.0 : 0.0; }

/* one dense layer: out[o] = b[o] + sum_i W[o][i] in[i] */
static void dense(const double* W, const double* b, int nout, int nin, const double* in, double* out) {
  for (int o = 0; o < nout; ++o) {
    double s = b[o];
    for (int i = 0; i < nin; ++i) s += W[o * nin + i] * in[i];
    out[o] = s;
  }
}

/* forward pass of one sample, keeping the pre-activations */
static void forward1(const double* w, const double* x, double z1[H], double z2[H], double z3[H], double y[2]) {
  double h[H];
  dense(w + OFF_W1, w + OFF_B1, H, OR_MLP_IN, x, z1);
  for (int k = 0; k < H; ++k) h[k] = or_relu(z1[k]);
  dense(w + OFF_W2, w + OFF_B2, H, H, h, z2);
  for (int k = 0; k < H; ++k) h[k] = or_relu(z2[k]);
  dense(w + OFF_W3, w + OFF_B3, H, H, h, z3);
  for (int k = 0; k < H; ++k) h[k] = or_relu(z3[k]);
  dense(w + OFF_W4, w + OFF_B4, OR_MLP_OUT, H, h, y);
}

void or_mlp_forward(const double* w, const double* X, long n, double* Y) {
#pragma omp parallel for
  for (long s = 0; s < n; ++s) {
    double z1[H], z2[H], z3[H];
    forward1(w, X + s * OR_MLP_IN, z1, z2, z3, Y + s * OR_MLP_OUT);
  }
}

double or_mlp_loss_grad(const double* w, const double* X, const double* Yt, long n, double* grad) {
  memset(grad, 0, sizeof(double) * OR_MLP_NPARAM);
  double loss = 0.0;
  for (long s = 0; s < n; ++s) {
    const double* x = X + s * OR_MLP_IN;
    double z1[H], z2[H], z3[H], y[OR_MLP_OUT];
    forward1(w, x, z1, z2, z3, y);
    double h1[H], h2[H], h3[H];
    for (int k = 0; k < H; ++k) {
      h1[k] = or_relu(z1[k]);
      h2[k] = or_relu(z2[k]);
      h3[k] = or_relu(z3[k]);
    }
    /* dL/dy */
    double dy[OR_MLP_OUT];
    for (int o = 0; o < OR_MLP_OUT; ++o) {
      const double r = y[o] - Yt[s * OR_MLP_OUT + o];
      loss += 0.5 * r * r / (double)n;
      dy[o] = r / (double)n;
    }
    /* output layer */
    double dh[H], dz[H];
    for (int o = 0; o < OR_MLP_OUT; ++o) {
      grad[OFF_B4 + o] += dy[o];
      for (int k = 0; k < H; ++k) grad[OFF_W4 + o * H + k] += dy[o] * h3[k];
    }
    for (int k = 0; k < H; ++k) {
      double t = 0.0;
      for (int o = 0; o < OR_MLP_OUT; ++o) t += w[OFF_W4 + o * H + k] * dy[o];
      dh[k] = t;
    }
    /* third layer */
    for (int k = 0; k < H; ++k) dz[k] = dh[k] * or_relu_d(z3[k]);
    for (int o = 0; o < H; ++o) {
      grad[OFF_B3 + o] += dz[o];
      for (int k = 0; k < H; ++k) grad[OFF_W3 + o * H + k] += dz[o] * h2[k];
    }
    for (int k = 0; k < H; ++k) {
      double t = 0.0;
      for (int o = 0; o < H; ++o) t += w[OFF_W3 + o * H + k] * dz[o];
      dh[k] = t;
    }
    /* second layer */
    for (int k = 0; k < H; ++k) dz[k] = dh[k] * or_relu_d(z2[k]);
    for (int o = 0; o < H; ++o) {
      grad[OFF_B2 + o] += dz[o];
      for (int k = 0; k < H; ++k) grad[OFF_W2 + o * H + k] += dz[o] * h1[k];
    }
    for (int k = 0; k < H; ++k) {
      double t = 0.0;
      for (int o = 0; o < H; ++o) t += w[OFF_W2 + o * H + k] * dz[o];
      dh[k] = t;
    }
    /* first layer */
    for (int k = 0; k < H; ++k) dz[k] = dh[k] * or_relu_d(z1[k]);
    for (int o = 0; o < H; ++o) {
      grad[OFF_B1 + o] += dz[o];
      for (int i = 0; i < OR_MLP_IN; ++i) grad[OFF_W1 + o * OR_MLP_IN + i] += dz[o] * x[i];
    }
  }
  return loss;
}

void or_adam_step(double* w, double* m, double* v, const double* g, long np, double lr, double b1, double b2,
                  double eps, int t) {
  const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (long k = 0; k < np; ++k) {
    m[k] = b1 * m[k] + (1.0 - b1) * g[k];
    v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
    const double mh = m[k] / c1, vh = v[k] / c2;
    w[k] -= lr * mh / (sqrt(vh) + eps);
  }
}

long or_mlp_nparam(void) { return OFF_END; }
