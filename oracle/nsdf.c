/* CPU oracle for the neural SDF surrogate.  TEST INFRASTRUCTURE ONLY.
 *
 * Network (per object): x_hat in [-1,1]^3 (the object's grid box mapped to the unit cube)
 *   -> positional encoding, 48 features ordered [sin(2^0 pi x) xyz, cos(2^0 pi x) xyz,
 *      sin(2^1 pi x) xyz, ..., cos(2^7 pi x) xyz]
 *   -> 4 hidden layers of width 64 with SiLU (z * sigmoid(z))
 *   -> 1 linear output; phi = half_extent * out.
 * Parameters (15681, flat): W1[64][48], b1[64], W2[64][64], b2[64], W3, b3, W4, b4, w5[64], b5.
 *
 * Loss: mean absolute error of out against phi_target / half_extent (L1).  Optimiser: Adam.
 * Everything in FP64; nsdf_forward_bf16 additionally rounds the GEMM operands (weights and the
 * activations entering each layer) to BF16, the way a BF16 MFMA path does.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <string.h>

#define NS_F 48
#define NS_H 64
#define NS_NPARAM (NS_H * NS_F + NS_H + 3 * (NS_H * NS_H + NS_H) + NS_H + 1)

float or_bf16_round(float x);

static double bf(double x, int on) { return on ? (double)or_bf16_round((float)x) : x; }

static void param_views(const double* P, const double** W, const double** b) {
  /* W[0..3], b[0..3] for the four hidden layers, W[4] = w5, b[4] = &b5 */
  const double* p = P;
  W[0] = p; p += NS_H * NS_F;
  b[0] = p; p += NS_H;
  for (int l = 1; l < 4; ++l) {
    W[l] = p; p += NS_H * NS_H;
    b[l] = p; p += NS_H;
  }
  W[4] = p; p += NS_H;
  b[4] = p;
}

int or_nsdf_num_params(void) { return NS_NPARAM; }

static void encode(const double* x, double* f) {
  for (int k = 0; k < 8; ++k) {
    const double w = ldexp(M_PI, k);
    for (int d = 0; d < 3; ++d) {
      f[6 * k + d] = sin(w * x[d]);
      f[6 * k + 3 + d] = cos(w * x[d]);
    }
  }
}

static double sigm(double z) { return 1.0 / (1.0 + exp(-z)); }

/* Forward for one point; keeps pre-activations z[4][64] and activations a[5][64] (a[0] = features). */
static double forward1(const double* P, const double* x, double z[4][NS_H], double a[5][NS_H], int bfl) {
  const double *W[5], *b[5];
  param_views(P, W, b);
  double f[NS_F];
  encode(x, f);
  for (int i = 0; i < NS_F; ++i) a[0][i] = f[i];
  int nin = NS_F;
  for (int l = 0; l < 4; ++l) {
    for (int o = 0; o < NS_H; ++o) {
      double s = 0;
      for (int i = 0; i < nin; ++i) s += bf(W[l][o * nin + i], bfl) * bf(a[l][i], bfl);
      s += b[l][o];
      z[l][o] = s;
      a[l + 1][o] = s * sigm(s);
    }
    nin = NS_H;
  }
  double out = b[4][0];
  for (int i = 0; i < NS_H; ++i) out += W[4][i] * a[4][i];
  return out;
}

/* out[n] and, if gx != NULL, d out / d x_hat [n][3] (reverse pass through the network). */
void or_nsdf_forward(const double* P, int64_t n, const double* x, double* out, double* gx, int bf16) {
  const double *W[5], *b[5];
  param_views(P, W, b);
  for (int64_t s = 0; s < n; ++s) {
    double z[4][NS_H], a[5][NS_H];
    out[s] = forward1(P, x + 3 * s, z, a, bf16);
    if (!gx) continue;
    double g[NS_H], gn[NS_H];
    for (int i = 0; i < NS_H; ++i) g[i] = W[4][i];          /* d out / d a4 */
    for (int l = 3; l >= 0; --l) {
      const int nin = l == 0 ? NS_F : NS_H;
      double dz[NS_H];
      for (int o = 0; o < NS_H; ++o) {
        const double sg = sigm(z[l][o]);
        dz[o] = g[o] * sg * (1.0 + z[l][o] * (1.0 - sg));
      }
      for (int i = 0; i < nin; ++i) {
        double t = 0;
        for (int o = 0; o < NS_H; ++o) t += W[l][o * nin + i] * dz[o];
        gn[i] = t;
      }
      for (int i = 0; i < nin; ++i) g[i] = gn[i];
    }
    /* through the encoding */
    for (int d = 0; d < 3; ++d) {
      double t = 0;
      for (int k = 0; k < 8; ++k) {
        const double w = ldexp(M_PI, k);
        t += g[6 * k + d] * w * cos(w * x[3 * s + d]) - g[6 * k + 3 + d] * w * sin(w * x[3 * s + d]);
      }
      gx[3 * s + d] = t;
    }
  }
}

/* Mean L1 loss over n points and its gradient with respect to every parameter (grad zeroed here). */
double or_nsdf_loss_grad(const double* P, int64_t n, const double* x, const double* target, double* grad) {
  const double *W[5], *b[5];
  param_views(P, W, b);
  double *GW[5], *Gb[5];
  param_views(grad, (const double**)GW, (const double**)Gb);
  memset(grad, 0, sizeof(double) * NS_NPARAM);
  double loss = 0;
  for (int64_t s = 0; s < n; ++s) {
    double z[4][NS_H], a[5][NS_H];
    const double out = forward1(P, x + 3 * s, z, a, 0);
    const double r = out - target[s];
    loss += fabs(r);
    const double go = (r > 0 ? 1.0 : (r < 0 ? -1.0 : 0.0)) / (double)n;
    Gb[4][0] += go;
    double g[NS_H];
    for (int i = 0; i < NS_H; ++i) {
      GW[4][i] += go * a[4][i];
      g[i] = go * W[4][i];
    }
    for (int l = 3; l >= 0; --l) {
      const int nin = l == 0 ? NS_F : NS_H;
      double dz[NS_H], gn[NS_H];
      for (int o = 0; o < NS_H; ++o) {
        const double sg = sigm(z[l][o]);
        dz[o] = g[o] * sg * (1.0 + z[l][o] * (1.0 - sg));
        Gb[l][o] += dz[o];
        for (int i = 0; i < nin; ++i) GW[l][o * nin + i] += dz[o] * a[l][i];
      }
      if (l > 0) {
        for (int i = 0; i < nin; ++i) {
          double t = 0;
          for (int o = 0; o < NS_H; ++o) t += W[l][o * nin + i] * dz[o];
          gn[i] = t;
        }
        for (int i = 0; i < nin; ++i) g[i] = gn[i];
      }
    }
  }
  return loss / (double)n;
}

/* One Adam step (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
void or_nsdf_adam(double* P, double* m, double* v, const double* g, int64_t np, int t, double lr, double b1, double b2,
                  double eps) {
  const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (int64_t i = 0; i < np; ++i) {
    m[i] = b1 * m[i] + (1 - b1) * g[i];
    v[i] = b2 * v[i] + (1 - b2) * g[i] * g[i];
    P[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}
