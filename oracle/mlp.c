/*
 * mlp.c -- FP64 reference of the small per-group rebuild predictor: a
 * 12-64-64-1 perceptron with tanh hidden layers and a logistic output,
 * trained on the mean binary cross-entropy, with the Adam update
 * (Kingma & Ba 2015).
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).  Plain loops in FP64; no code is
 * shared with the GPU kernels.
 *
 * Parameter vector (MLP_NPARAM doubles, this order):
 *   W1 [64][12] row-major, b1 [64], W2 [64][64] row-major, b2 [64],
 *   w3 [64], b3 [1].
 *   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), p = 1 / (1 + exp(-(w3.h2 + b3)))
 *   loss = -(1/n) sum_i [w y_i log p_i + (1 - y_i) log(1 - p_i)],
 *   w = pos_weight (1 for the plain cross-entropy)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NIN 12
#define NH 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NIN)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NH)
#define MLP_NPARAM (OFF_B3 + 1)

int orc_mlp_nparam(void) { return MLP_NPARAM; }

static void forward_one(const double* w, const double* x, double* h1,
                        double* h2, double* p) {
  for (int j = 0; j < NH; ++j) {
    double s = w[OFF_B1 + j];
    for (int k = 0; k < NIN; ++k) s += w[OFF_W1 + j * NIN + k] * x[k];
    h1[j] = tanh(s);
  }
  for (int j = 0; j < NH; ++j) {
    double s = w[OFF_B2 + j];
    for (int k = 0; k < NH; ++k) s += w[OFF_W2 + j * NH + k] * h1[k];
    h2[j] = tanh(s);
  }
  double z = w[OFF_B3];
  for (int k = 0; k < NH; ++k) z += w[OFF_W3 + k] * h2[k];
  *p = 1.0 / (1.0 + exp(-z));
}

int orc_mlp_forward(const double* w, int64_t n, const double* x, double* p) {
  if (!w || n < 0 || (n > 0 && (!x || !p))) return -1;
  double h1[NH], h2[NH];
  for (int64_t i = 0; i < n; ++i) forward_one(w, x + NIN * i, h1, h2, &p[i]);
  return 0;
}

/* Mean cross-entropy and its gradient by back-propagation. */
int orc_mlp_loss_grad(const double* w, int64_t n, const double* x,
                      const double* y, double pos_weight, double* loss,
                      double* grad) {
  if (!w || n <= 0 || !x || !y || !loss || !grad || !(pos_weight > 0.0))
    return -1;
  memset(grad, 0, sizeof(double) * MLP_NPARAM);
  double h1[NH], h2[NH], d2[NH], d1[NH], p;
  double L = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double* xi = x + NIN * i;
    forward_one(w, xi, h1, h2, &p);
    const double pc = p < 1e-300 ? 1e-300 : (p > 1.0 - 1e-16 ? 1.0 - 1e-16 : p);
    L -= pos_weight * y[i] * log(pc) + (1.0 - y[i]) * log(1.0 - pc);
    /* dL/dz of the weighted cross-entropy through the logistic output:
     * p (w y + 1 - y) - w y  (= p - y when w = 1) */
    const double wy = pos_weight * y[i];
    const double dz = (p * (wy + 1.0 - y[i]) - wy) / (double)n;
    grad[OFF_B3] += dz;
    for (int k = 0; k < NH; ++k) {
      grad[OFF_W3 + k] += dz * h2[k];
      d2[k] = dz * w[OFF_W3 + k] * (1.0 - h2[k] * h2[k]);
    }
    for (int j = 0; j < NH; ++j) {
      grad[OFF_B2 + j] += d2[j];
      for (int k = 0; k < NH; ++k) grad[OFF_W2 + j * NH + k] += d2[j] * h1[k];
    }
    for (int k = 0; k < NH; ++k) {
      double s = 0.0;
      for (int j = 0; j < NH; ++j) s += d2[j] * w[OFF_W2 + j * NH + k];
      d1[k] = s * (1.0 - h1[k] * h1[k]);
    }
    for (int j = 0; j < NH; ++j) {
      grad[OFF_B1 + j] += d1[j];
      for (int k = 0; k < NIN; ++k) grad[OFF_W1 + j * NIN + k] += d1[j] * xi[k];
    }
  }
  *loss = L / (double)n;
  return 0;
}

/* One Adam update of step t (t >= 1) with moments m, v (updated in place). */
int orc_adam(double* w, const double* g, double* m, double* v, int64_t t,
             double lr, double beta1, double beta2, double eps) {
  if (!w || !g || !m || !v || t < 1) return -1;
  const double c1 = 1.0 - pow(beta1, (double)t);
  const double c2 = 1.0 - pow(beta2, (double)t);
  for (int k = 0; k < MLP_NPARAM; ++k) {
    m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
    v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
    const double mh = m[k] / c1;
    const double vh = v[k] / c2;
    w[k] -= lr * mh / (sqrt(vh) + eps);
  }
  return 0;
}
