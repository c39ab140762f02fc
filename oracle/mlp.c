/*
 * mlp.c -- FP64 oracle of the muscle-geometry surrogate network (TEST
 * INFRASTRUCTURE; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it).
 *
 * Network: x (n0) -> SiLU(W1 x + b1) (n1) -> SiLU(W2 h1 + b2) (n2) ->
 * W3 h2 + b3 (n3). Weights are stored row-major as W[in][out] (y = x W + b).
 * The GPU multiplies bfloat16 operands with float32 accumulation; this
 * oracle rounds the same operands to bfloat16 (round to nearest even) at the
 * same points when `bf16` is set, and accumulates in double. With `bf16`
 * unset it is the plain FP64 network (used for finite-difference checks).
 *
 * Loss: mean over (sample, output) of mask * (y - t)^2, i.e.
 * L = sum(mask (y - t)^2) / (B * n3), so dL/dy = 2 mask (y - t) / (B n3).
 * Adam: Kingma & Ba (2015) with bias correction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* round a float to bfloat16 (nearest even) and back */
double ora_bf16(double v) {
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) { /* inf / nan */
    if (u & 0x007FFFFFu) u |= 0x00400000u;
    u &= 0xFFFF0000u;
  } else {
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
  }
  memcpy(&f, &u, 4);
  return (double)f;
}

static double rnd(double v, int bf16) { return bf16 ? ora_bf16(v) : v; }
static double sigm(double z) { return 1.0 / (1.0 + exp(-z)); }
static double silu(double z) { return z * sigm(z); }
static double silu_d(double z) {
  double s = sigm(z);
  return s * (1.0 + z * (1.0 - s));
}

/* y = x W + b for one layer: x [B][n], W [n][m] (weights already rounded) */
/* Each output is 0 + x_0 W_0j + x_1 W_1j + ... (i ascending), then + b_j;
 * the loops run i before j only so that W is read row by row. */
static void affine(int B, int n, int m, const double *x, const double *W, const float *b,
                   double *y) {
  for (int s = 0; s < B; ++s) {
    double *ys = y + (size_t)s * m;
    for (int j = 0; j < m; ++j) ys[j] = 0.0;
    for (int i = 0; i < n; ++i) {
      const double xi = x[(size_t)s * n + i];
      const double *Wi = W + (size_t)i * m;
      for (int j = 0; j < m; ++j) ys[j] += xi * Wi[j];
    }
    for (int j = 0; j < m; ++j) ys[j] += (double)b[j];
  }
}

/* gW[i][j] = sum over samples b (ascending) of a[b][i] d[b][j], summed in
 * that order from 0; the loops run over b outermost only so that the rows
 * are read contiguously. */
static void outer_sum(int B, int n, int m, const double *a, const double *d, double *gW) {
  for (size_t k = 0; k < (size_t)n * m; ++k) gW[k] = 0.0;
  for (int b = 0; b < B; ++b)
    for (int i = 0; i < n; ++i) {
      const double ai = a[(size_t)b * n + i];
      const double *db = d + (size_t)b * m;
      double *g = gW + (size_t)i * m;
      for (int j = 0; j < m; ++j) g[j] += ai * db[j];
    }
}

static double *rounded(const float *w, size_t n, int bf16) {
  double *o = (double *)malloc(sizeof(double) * (n ? n : 1));
  for (size_t i = 0; i < n; ++i) o[i] = rnd((double)w[i], bf16);
  return o;
}

/* Forward pass. z1, h1, z2, h2 (optional, may be NULL) receive the
 * pre-activations and the activations as fed to the next layer (rounded). */
void ora_mlp_forward(int B, int n0, int n1, int n2, int n3, const float *W1, const float *b1,
                     const float *W2, const float *b2, const float *W3, const float *b3,
                     const float *x, int bf16, double *y, double *z1o, double *h1o,
                     double *z2o, double *h2o) {
  double *w1 = rounded(W1, (size_t)n0 * n1, bf16), *w2 = rounded(W2, (size_t)n1 * n2, bf16),
         *w3 = rounded(W3, (size_t)n2 * n3, bf16);
  double *xr = rounded(x, (size_t)B * n0, bf16);
  double *z1 = (double *)malloc(sizeof(double) * B * n1), *h1 = (double *)malloc(sizeof(double) * B * n1);
  double *z2 = (double *)malloc(sizeof(double) * B * n2), *h2 = (double *)malloc(sizeof(double) * B * n2);
  affine(B, n0, n1, xr, w1, b1, z1);
  for (size_t i = 0; i < (size_t)B * n1; ++i) h1[i] = rnd(silu(z1[i]), bf16);
  affine(B, n1, n2, h1, w2, b2, z2);
  for (size_t i = 0; i < (size_t)B * n2; ++i) h2[i] = rnd(silu(z2[i]), bf16);
  affine(B, n2, n3, h2, w3, b3, y);
  if (z1o) memcpy(z1o, z1, sizeof(double) * B * n1);
  if (h1o) memcpy(h1o, h1, sizeof(double) * B * n1);
  if (z2o) memcpy(z2o, z2, sizeof(double) * B * n2);
  if (h2o) memcpy(h2o, h2, sizeof(double) * B * n2);
  free(w1); free(w2); free(w3); free(xr); free(z1); free(h1); free(z2); free(h2);
}

/* Loss and gradients of all parameters (float64 outputs, same layouts).
 * Backward matmul operands (dy, dz, W, activations) are rounded to
 * bfloat16 when bf16 is set, as on the GPU. Returns the loss. */
double ora_mlp_grad(int B, int n0, int n1, int n2, int n3, const float *W1, const float *b1,
                    const float *W2, const float *b2, const float *W3, const float *b3,
                    const float *x, const float *t, const float *mask, int bf16, double *gW1,
                    double *gb1, double *gW2, double *gb2, double *gW3, double *gb3) {
  double *y = (double *)malloc(sizeof(double) * B * n3);
  double *z1 = (double *)malloc(sizeof(double) * B * n1), *h1 = (double *)malloc(sizeof(double) * B * n1);
  double *z2 = (double *)malloc(sizeof(double) * B * n2), *h2 = (double *)malloc(sizeof(double) * B * n2);
  ora_mlp_forward(B, n0, n1, n2, n3, W1, b1, W2, b2, W3, b3, x, bf16, y, z1, h1, z2, h2);
  double *w2 = rounded(W2, (size_t)n1 * n2, bf16), *w3 = rounded(W3, (size_t)n2 * n3, bf16);
  double *xr = rounded(x, (size_t)B * n0, bf16);
  double *dy = (double *)malloc(sizeof(double) * B * n3);
  double *dz2 = (double *)malloc(sizeof(double) * B * n2), *dz1 = (double *)malloc(sizeof(double) * B * n1);
  const double scale = 2.0 / ((double)B * n3);
  double loss = 0.0;
  for (size_t i = 0; i < (size_t)B * n3; ++i) {
    double m = mask ? (double)mask[i] : 1.0;
    double d = y[i] - (double)t[i];
    loss += m * d * d;
    dy[i] = m * scale * d;
  }
  loss /= (double)B * n3;
  /* layer 3 */
  for (int j = 0; j < n3; ++j) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += dy[(size_t)b * n3 + j];
    gb3[j] = s;
  }
  for (size_t i = 0; i < (size_t)B * n3; ++i) dy[i] = rnd(dy[i], bf16);
  outer_sum(B, n2, n3, h2, dy, gW3);
  for (int b = 0; b < B; ++b)
    for (int i = 0; i < n2; ++i) {
      double s = 0.0;
      for (int j = 0; j < n3; ++j) s += dy[(size_t)b * n3 + j] * w3[(size_t)i * n3 + j];
      dz2[(size_t)b * n2 + i] = s * silu_d(z2[(size_t)b * n2 + i]);
    }
  /* layer 2 */
  for (int j = 0; j < n2; ++j) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += dz2[(size_t)b * n2 + j];
    gb2[j] = s;
  }
  for (size_t i = 0; i < (size_t)B * n2; ++i) dz2[i] = rnd(dz2[i], bf16);
  outer_sum(B, n1, n2, h1, dz2, gW2);
  for (int b = 0; b < B; ++b)
    for (int i = 0; i < n1; ++i) {
      double s = 0.0;
      for (int j = 0; j < n2; ++j) s += dz2[(size_t)b * n2 + j] * w2[(size_t)i * n2 + j];
      dz1[(size_t)b * n1 + i] = s * silu_d(z1[(size_t)b * n1 + i]);
    }
  /* layer 1 */
  for (int j = 0; j < n1; ++j) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += dz1[(size_t)b * n1 + j];
    gb1[j] = s;
  }
  for (size_t i = 0; i < (size_t)B * n1; ++i) dz1[i] = rnd(dz1[i], bf16);
  outer_sum(B, n0, n1, xr, dz1, gW1);
  free(y); free(z1); free(h1); free(z2); free(h2); free(w2); free(w3); free(xr); free(dy);
  free(dz2); free(dz1);
  return loss;
}

/* One Adam step on n parameters (double state). step = t >= 1. */
void ora_adam(int n, double *w, double *m, double *v, const double *g, double lr, double b1,
              double b2, double eps, int step) {
  double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (int i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    w[i] -= lr * mh / (sqrt(vh) + eps);
  }
}
