/*
 * FP64 oracle of the search-bracket MLP — TEST INFRASTRUCTURE ONLY.
 *
 * The network maps D input features to one output through two hidden
 * layers of H units with ReLU:
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), out = w3 . h2 + b3,
 * and is trained with the Huber loss (quadratic within delta of the target,
 * linear beyond). It is not part of the paper's method; it only seeds the
 * decoder's search, whose result is verified against the exact CDF.
 * Parameters are one flat array: W1 [H][D], b1 [H], W2 [H][H], b2 [H],
 * w3 [H], b3 [1]. Loss and gradients are sums over the samples.
 *
 * With round_act the first hidden layer's activations relu(W1 x + b1) are
 * rounded to bfloat16 (the 8-significant-bit format the decoder's matrix
 * cores read: the value rounded to binary32, then its low 16 bits rounded
 * off to nearest, ties to even) before the second layer uses them, and the
 * gradient passes through the rounding unchanged (straight-through): the
 * mask of the first layer is still "pre-activation > 0".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double bf16_round(double v) {
  float f = (float)v;
  uint32_t b;
  memcpy(&b, &f, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  b &= 0xFFFF0000u;
  memcpy(&f, &b, 4);
  return (double)f;
}

static int64_t n_params(int D, int H) { return (int64_t)H * D + H + (int64_t)H * H + H + H + 1; }

int64_t gmm_oracle_mlp_num_params(int32_t D, int32_t H) { return n_params(D, H); }

/* Forward pass of one sample; fills the pre-activations z1, z2 (length H)
 * and the first layer's activations a1 (rounded with round_act), and
 * returns the output. */
static double forward1(int D, int H, const double* p, const double* x, int round_act, double* z1,
                       double* a1, double* z2) {
  const double* W1 = p;
  const double* b1 = W1 + (int64_t)H * D;
  const double* W2 = b1 + H;
  const double* b2 = W2 + (int64_t)H * H;
  const double* w3 = b2 + H;
  const double b3 = w3[H];
  for (int h = 0; h < H; ++h) {
    double s = b1[h];
    for (int d = 0; d < D; ++d) s += W1[(int64_t)h * D + d] * x[d];
    z1[h] = s;
    const double a = s > 0.0 ? s : 0.0;
    a1[h] = round_act ? bf16_round(a) : a;
  }
  for (int h = 0; h < H; ++h) {
    double s = b2[h];
    for (int k = 0; k < H; ++k) s += W2[(int64_t)h * H + k] * a1[k];
    z2[h] = s;
  }
  double out = b3;
  for (int h = 0; h < H; ++h) out += w3[h] * (z2[h] > 0.0 ? z2[h] : 0.0);
  return out;
}

void gmm_oracle_mlp_forward(int32_t D, int32_t H, const double* params, int64_t n,
                            const double* X, int32_t round_act, double* out) {
  double* z = (double*)malloc(sizeof(double) * 3 * (size_t)H);
  for (int64_t i = 0; i < n; ++i)
    out[i] = forward1(D, H, params, X + i * D, round_act, z, z + H, z + 2 * H);
  free(z);
}

/* Sum over samples of the Huber loss of (out - y) and its gradient with
 * respect to every parameter (grad has the parameter layout). */
double gmm_oracle_mlp_loss_grad(int32_t D, int32_t H, const double* params, int64_t n,
                                const double* X, const double* y, double delta,
                                int32_t round_act, double* grad) {
  const int64_t P = n_params(D, H);
  memset(grad, 0, sizeof(double) * (size_t)P);
  double* gW1 = grad;
  double* gb1 = gW1 + (int64_t)H * D;
  double* gW2 = gb1 + H;
  double* gb2 = gW2 + (int64_t)H * H;
  double* gw3 = gb2 + H;
  double* gb3 = gw3 + H;
  const double* W2 = params + (int64_t)H * D + H;
  const double* w3 = W2 + (int64_t)H * H + H;
  double* buf = (double*)malloc(sizeof(double) * 5 * (size_t)H);
  double *z1 = buf, *z2 = buf + H, *d2 = buf + 2 * H, *d1 = buf + 3 * H, *a1 = buf + 4 * H;
  double loss = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double* x = X + i * D;
    const double out = forward1(D, H, params, x, round_act, z1, a1, z2);
    const double r = out - y[i];
    const double ar = fabs(r);
    loss += (ar <= delta) ? 0.5 * r * r : delta * (ar - 0.5 * delta);
    const double g = (ar <= delta) ? r : (r > 0 ? delta : -delta);
    *gb3 += g;
    for (int h = 0; h < H; ++h) {
      const double a2 = z2[h] > 0.0 ? z2[h] : 0.0;
      gw3[h] += g * a2;
      d2[h] = (z2[h] > 0.0) ? g * w3[h] : 0.0;
    }
    for (int h = 0; h < H; ++h) {
      gb2[h] += d2[h];
      for (int k = 0; k < H; ++k) gW2[(int64_t)h * H + k] += d2[h] * a1[k];
    }
    for (int k = 0; k < H; ++k) {
      double s = 0.0;
      for (int h = 0; h < H; ++h) s += d2[h] * W2[(int64_t)h * H + k];
      d1[k] = (z1[k] > 0.0) ? s : 0.0;
    }
    for (int h = 0; h < H; ++h) {
      gb1[h] += d1[h];
      for (int d = 0; d < D; ++d) gW1[(int64_t)h * D + d] += d1[h] * x[d];
    }
  }
  free(buf);
  return loss;
}
