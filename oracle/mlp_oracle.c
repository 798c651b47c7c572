/* mlp_oracle.c -- TEST INFRASTRUCTURE ONLY: a plain FP64 reference of the
 * small multilayer perceptron that predicts per-level truncation errors for
 * the learned-order mode, with its loss gradient and the Adam update.
 *
 * Network: 3 inputs -> 64 ReLU -> 64 ReLU -> 21 linear outputs.
 * Parameters, one flat array (row-major, output index major):
 *   W1[64][3], b1[64], W2[64][64], b2[64], W3[21][64], b3[21]   (5781 values)
 * Loss over a batch of m samples x[m][3] with targets t[m][21]:
 *   loss = (1 / (21 m)) sum_{i,o} (y_io - t_io)^2
 * Gradient by the chain rule (backpropagation), layer by layer.
 * Adam: Kingma and Ba, "Adam: a method for stochastic optimization" (ICLR
 * 2015), Algorithm 1, with bias-corrected first and second moments.
 * Nothing here is shared with the GPU path. */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define NI 3
#define NH 64
#define NO 21
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NI)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NO * NH)
#define NPARAM (OFF_B3 + NO)

int oracle_mlp_nparam(void) { return NPARAM; }

/* One sample: pre-activations z1, z2, activations h1, h2 and outputs y. */
static void forward_one(const double* w, const double* x, double* z1, double* h1, double* z2,
                        double* h2, double* y) {
  for (int j = 0; j < NH; ++j) {
    double s = w[OFF_B1 + j];
    for (int i = 0; i < NI; ++i) s += w[OFF_W1 + j * NI + i] * x[i];
    z1[j] = s;
    h1[j] = s > 0 ? s : 0;
  }
  for (int j = 0; j < NH; ++j) {
    double s = w[OFF_B2 + j];
    for (int i = 0; i < NH; ++i) s += w[OFF_W2 + j * NH + i] * h1[i];
    z2[j] = s;
    h2[j] = s > 0 ? s : 0;
  }
  for (int o = 0; o < NO; ++o) {
    double s = w[OFF_B3 + o];
    for (int i = 0; i < NH; ++i) s += w[OFF_W3 + o * NH + i] * h2[i];
    y[o] = s;
  }
}

void oracle_mlp_forward(const double* w, int64_t m, const double* x, double* y) {
  double z1[NH], h1[NH], z2[NH], h2[NH];
  for (int64_t s = 0; s < m; ++s) forward_one(w, x + NI * s, z1, h1, z2, h2, y + NO * s);
}

/* Returns the loss; g receives d loss / d w (NPARAM values). */
double oracle_mlp_loss_grad(const double* w, int64_t m, const double* x, const double* t,
                            double* g) {
  memset(g, 0, sizeof(double) * NPARAM);
  double loss = 0;
  const double scale = 1.0 / (double)(NO * (m > 0 ? m : 1));
  for (int64_t s = 0; s < m; ++s) {
    double z1[NH], h1[NH], z2[NH], h2[NH], y[NO];
    const double* xs = x + NI * s;
    forward_one(w, xs, z1, h1, z2, h2, y);
    double dy[NO], dh2[NH], dz2[NH], dh1[NH], dz1[NH];
    for (int o = 0; o < NO; ++o) {
      const double e = y[o] - t[NO * s + o];
      loss += e * e;
      dy[o] = 2.0 * e * scale;
    }
    /* output layer */
    for (int o = 0; o < NO; ++o) {
      g[OFF_B3 + o] += dy[o];
      for (int i = 0; i < NH; ++i) g[OFF_W3 + o * NH + i] += dy[o] * h2[i];
    }
    for (int i = 0; i < NH; ++i) {
      double a = 0;
      for (int o = 0; o < NO; ++o) a += w[OFF_W3 + o * NH + i] * dy[o];
      dh2[i] = a;
      dz2[i] = z2[i] > 0 ? a : 0;
    }
    /* second hidden layer */
    for (int j = 0; j < NH; ++j) {
      g[OFF_B2 + j] += dz2[j];
      for (int i = 0; i < NH; ++i) g[OFF_W2 + j * NH + i] += dz2[j] * h1[i];
    }
    for (int i = 0; i < NH; ++i) {
      double a = 0;
      for (int j = 0; j < NH; ++j) a += w[OFF_W2 + j * NH + i] * dz2[j];
      dh1[i] = a;
      dz1[i] = z1[i] > 0 ? a : 0;
    }
    /* first hidden layer */
    for (int j = 0; j < NH; ++j) {
      g[OFF_B1 + j] += dz1[j];
      for (int i = 0; i < NI; ++i) g[OFF_W1 + j * NI + i] += dz1[j] * xs[i];
    }
    (void)dh1;
    (void)dh2;
  }
  return loss * scale;
}

/* One Adam step (step counts from 1). */
void oracle_mlp_adam(int64_t n, double* w, const double* g, double* m1, double* m2, int step,
                     double lr, double beta1, double beta2, double eps) {
  const double c1 = 1.0 - pow(beta1, (double)step);
  const double c2 = 1.0 - pow(beta2, (double)step);
  for (int64_t i = 0; i < n; ++i) {
    m1[i] = beta1 * m1[i] + (1.0 - beta1) * g[i];
    m2[i] = beta2 * m2[i] + (1.0 - beta2) * g[i] * g[i];
    const double mh = m1[i] / c1, vh = m2[i] / c2;
    w[i] -= lr * mh / (sqrt(vh) + eps);
  }
}
