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
 * Everything in FP64.  With bf16 = 1 the forward emulates a BF16 MFMA path: weights and the
 * activations entering each layer are rounded to BF16, the layer sum (bias included) is kept
 * wide, and the pre-activation is rounded to BF16 before SiLU (activations are BF16 tensors).
 * The oracle's own weights, sums and reverse-pass bookkeeping are FP64 throughout.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdlib.h>
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

/* Forward for one point; keeps pre-activations z[4][64] and activations a[5][64] (a[0] = features).
 * zw (or NULL) records each layer sum before its BF16 rounding and sabs the sum of the absolute
 * values of its terms (bias included): what the rounding of z acted on, and its scale. */
static double forward1t(const double* P, const double* x, double z[4][NS_H], double a[5][NS_H], int bfl,
                        double zw[4][NS_H], double sabs[4][NS_H]) {
  const double *W[5], *b[5];
  param_views(P, W, b);
  double f[NS_F];
  encode(x, f);
  for (int i = 0; i < NS_F; ++i) a[0][i] = f[i];
  int nin = NS_F;
  for (int l = 0; l < 4; ++l) {
    for (int o = 0; o < NS_H; ++o) {
      double s = 0, sa = 0;
      for (int i = 0; i < nin; ++i) {
        const double t = bf(W[l][o * nin + i], bfl) * bf(a[l][i], bfl);
        s += t;
        sa += fabs(t);
      }
      s += b[l][o];
      if (zw) {
        zw[l][o] = s;
        sabs[l][o] = sa + fabs(b[l][o]);
      }
      s = bf(s, bfl);
      z[l][o] = s;
      a[l + 1][o] = s * sigm(s);
    }
    nin = NS_H;
  }
  double out = b[4][0];
  for (int i = 0; i < NS_H; ++i) out += W[4][i] * a[4][i];
  return out;
}

static double forward1(const double* P, const double* x, double z[4][NS_H], double a[5][NS_H], int bfl) {
  return forward1t(P, x, z, a, bfl, NULL, NULL);
}

/* The BF16-rounding record of the forward pass at n points (diagnostics of BF16 rounding ties):
 * feat[n][48] the encoding features before rounding, zw[n][4][64] the layer sums before rounding,
 * zb[n][4][64] after it (the pre-activations SiLU sees), sabs[n][4][64] the sum of the absolute
 * values of each layer sum's terms.  bf16 = 1 is the BF16-emulating network. */
void or_nsdf_forward_trace(const double* P, int64_t n, const double* x, double* feat, double* zw, double* zb,
                           double* sabs, int bf16) {
  for (int64_t s = 0; s < n; ++s) {
    double z[4][NS_H], a[5][NS_H], w[4][NS_H], sa[4][NS_H];
    (void)forward1t(P, x + 3 * s, z, a, bf16, w, sa);
    for (int i = 0; i < NS_F; ++i) feat[s * NS_F + i] = a[0][i];
    for (int l = 0; l < 4; ++l)
      for (int o = 0; o < NS_H; ++o) {
        const int64_t k = (s * 4 + l) * NS_H + o;
        zw[k] = w[l][o];
        zb[k] = z[l][o];
        sabs[k] = sa[l][o];
      }
  }
}

/* out[n] and, if gx != NULL, d out / d x_hat [n][3] (reverse pass through the network).  With
 * bf16 = 1 the reverse pass rounds its GEMM operands (weights and dz) to BF16 as well; the
 * output weights w5, the running gradient and the encoding derivative stay wide. */
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
        dz[o] = bf(g[o] * sg * (1.0 + z[l][o] * (1.0 - sg)), bf16);
      }
      for (int i = 0; i < nin; ++i) {
        double t = 0;
        for (int o = 0; o < NS_H; ++o) t += bf(W[l][o * nin + i], bf16) * dz[o];
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

/* silu' and silu'' at z (s = sigmoid(z)):  s (1 + z (1 - s))  and  s (1 - s) (2 + z (1 - 2 s)). */
static double dsilu(double z) {
  const double sg = sigm(z);
  return sg * (1.0 + z * (1.0 - sg));
}
static double d2silu(double z) {
  const double sg = sigm(z);
  return sg * (1.0 - sg) * (2.0 + z * (1.0 - 2.0 * sg));
}

/* Forward-mode tangent of one point along the input direction u (x_hat units), on top of the
 * primal pre-activations z of forward1: adot[0] = J_enc(x) u (the encoding's derivative along u),
 * zdot[l] = W_l adot[l] (no bias), adot[l+1] = silu'(z[l]) zdot[l].  Returns w5 . adot[4], the
 * directional derivative of out along u.  With bf16 = 1 the rounding follows the MFMA path: the
 * GEMM operands (adot[0..3], weights) and zdot are BF16; adot[4] feeds the FP32 output layer. */
static double tangent1(const double* P, const double* x, const double* u, double z[4][NS_H],
                       double zdot[4][NS_H], double adot[5][NS_H], int bfl) {
  const double *W[5], *b[5];
  param_views(P, W, b);
  for (int k = 0; k < 8; ++k) {
    const double w = ldexp(M_PI, k);
    for (int d = 0; d < 3; ++d) {
      adot[0][6 * k + d] = bf(w * cos(w * x[d]) * u[d], bfl);
      adot[0][6 * k + 3 + d] = bf(-w * sin(w * x[d]) * u[d], bfl);
    }
  }
  int nin = NS_F;
  for (int l = 0; l < 4; ++l) {
    for (int o = 0; o < NS_H; ++o) {
      double s = 0;
      for (int i = 0; i < nin; ++i) s += bf(W[l][o * nin + i], bfl) * adot[l][i];
      zdot[l][o] = bf(s, bfl);
      const double ad = dsilu(z[l][o]) * zdot[l][o];
      adot[l + 1][o] = l < 3 ? bf(ad, bfl) : ad;
    }
    nin = NS_H;
  }
  double h = 0;
  for (int i = 0; i < NS_H; ++i) h += W[4][i] * adot[4][i];
  return h;
}

/* Directional derivative of out along u[n][3] at every point by the tangent pass (dd[n]). */
void or_nsdf_dirderiv(const double* P, int64_t n, const double* x, const double* u, double* dd, int bf16) {
  for (int64_t s = 0; s < n; ++s) {
    double z[4][NS_H], a[5][NS_H], zdot[4][NS_H], adot[5][NS_H];
    (void)forward1(P, x + 3 * s, z, a, bf16);
    dd[s] = tangent1(P, x + 3 * s, u + 3 * s, z, zdot, adot, bf16);
  }
}

/* Loss over n points and its gradient with respect to every parameter (grad zeroed here):
 *   mean_i |out_i - t_i|                                               (L1 on the value)
 *   + pair_lambda * sum over pairs |(out_2i+1 - out_2i) - (t_2i+1 - t_2i)| / n      (n even)
 *   + grad_lambda * mean_i sum_d |g_i,d - gt_i,d|                      (L1 on the gradient)
 * with g_i = d out / d x_hat at x_i (the reverse pass of or_nsdf_forward) and gt[n][3] its
 * target (the grid's d phi / d q, which is d(phi/e) / d x_hat).  The pair term is a first-order
 * handle on the slope between nearby points; the gradient term supervises the slope itself.
 * Parameter gradient of the gradient term: with u_i = grad_lambda sign(g_i - gt_i) / n held
 * fixed it is the parameter gradient of u_i . g_i, the directional derivative of out along u_i,
 * which the tangent pass (tangent1) computes as w5 . adot_4.  Backpropagating through both the
 * primal and the tangent chain gives, per layer (abar, adbar the adjoints of a and adot):
 *   zdbar = adbar silu'(z);   zbar = abar silu'(z) + adbar silu''(z) zdot
 *   dW += zbar a_in^T + zdbar adot_in^T;   db += zbar;   abar_in = W^T zbar;  adbar_in = W^T zdbar
 * starting from abar_4 = go w5 (go = d loss / d out) and adbar_4 = w5, and dw5 += go a_4 + adot_4.
 * bf16 = 1 emulates the BF16 MFMA backward: every GEMM operand rounded to BF16 (zbar, zdbar,
 * the layer inputs a and adot, the weights); the output layer and all sums stay wide. */
double or_nsdf_loss_grad2(const double* P, int64_t n, const double* x, const double* target, const double* gtarget,
                          double* grad, int bf16, double pair_lambda, double grad_lambda) {
  const double *W[5], *b[5];
  param_views(P, W, b);
  double *GW[5], *Gb[5];
  param_views(grad, (const double**)GW, (const double**)Gb);
  memset(grad, 0, sizeof(double) * NS_NPARAM);
  const int gs = grad_lambda > 0 && gtarget != NULL;
  double loss = 0;
  double* res = NULL;   // residuals out - t of every point, for the pair term
  if (pair_lambda > 0) {
    res = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t s = 0; s < n; ++s) {
      double z[4][NS_H], a[5][NS_H];
      res[s] = forward1(P, x + 3 * s, z, a, bf16) - target[s];
    }
  }
  for (int64_t s = 0; s < n; ++s) {
    double z[4][NS_H], a[5][NS_H];
    const double out = forward1(P, x + 3 * s, z, a, bf16);
    const double r = out - target[s];
    loss += fabs(r);
    double go = (r > 0 ? 1.0 : (r < 0 ? -1.0 : 0.0)) / (double)n;
    if (pair_lambda > 0) {
      // d/d out_s of lambda |r_odd - r_even| is lambda * sign(r_s - r_partner) for both members
      const double dr = r - res[s ^ 1];
      go += pair_lambda * (dr > 0 ? 1.0 : (dr < 0 ? -1.0 : 0.0)) / (double)n;
      if ((s & 1) == 0) loss += pair_lambda * fabs(dr);
    }
    double zdot[4][NS_H], adot[5][NS_H];
    if (gs) {
      double o1, g[3], u[3];
      or_nsdf_forward(P, 1, x + 3 * s, &o1, g, bf16);
      for (int d = 0; d < 3; ++d) {
        const double e = g[d] - gtarget[3 * s + d];
        loss += grad_lambda * fabs(e);
        u[d] = grad_lambda * (e > 0 ? 1.0 : (e < 0 ? -1.0 : 0.0)) / (double)n;
      }
      (void)tangent1(P, x + 3 * s, u, z, zdot, adot, bf16);
    }
    Gb[4][0] += go;
    double ab[NS_H], adb[NS_H];
    for (int i = 0; i < NS_H; ++i) {
      GW[4][i] += go * a[4][i] + (gs ? adot[4][i] : 0.0);
      ab[i] = go * W[4][i];
      adb[i] = W[4][i];
    }
    for (int l = 3; l >= 0; --l) {
      const int nin = l == 0 ? NS_F : NS_H;
      double zb[NS_H], zdb[NS_H], gn[NS_H], gdn[NS_H];
      for (int o = 0; o < NS_H; ++o) {
        const double sg = sigm(z[l][o]);
        const double t1 = ab[o] * sg * (1.0 + z[l][o] * (1.0 - sg));   // abar silu'(z)
        zb[o] = bf(gs ? t1 + adb[o] * d2silu(z[l][o]) * zdot[l][o] : t1, bf16);
        zdb[o] = gs ? bf(adb[o] * dsilu(z[l][o]), bf16) : 0.0;
        Gb[l][o] += zb[o];
        for (int i = 0; i < nin; ++i) {
          GW[l][o * nin + i] += zb[o] * bf(a[l][i], bf16);
          if (gs) GW[l][o * nin + i] += zdb[o] * adot[l][i];
        }
      }
      if (l > 0) {
        for (int i = 0; i < nin; ++i) {
          double t = 0, td = 0;
          for (int o = 0; o < NS_H; ++o) {
            const double w = bf(W[l][o * nin + i], bf16);
            t += w * zb[o];
            td += w * zdb[o];
          }
          gn[i] = t;
          gdn[i] = td;
        }
        for (int i = 0; i < nin; ++i) {
          ab[i] = gn[i];
          adb[i] = gdn[i];
        }
      }
    }
  }
  free(res);
  return loss / (double)n;
}

/* The loss and gradient without the gradient term. */
double or_nsdf_loss_grad(const double* P, int64_t n, const double* x, const double* target, double* grad, int bf16,
                         double pair_lambda) {
  return or_nsdf_loss_grad2(P, n, x, target, NULL, grad, bf16, pair_lambda, 0.0);
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

/* Training targets in FP64: the point is clamped into the node-centred grid box
 * [origin, origin + (n-1) h]^3, phi is the trilinear interpolant of the grid samples there
 * (App. A.1, sdf backend), and the record is { (q - c) / e, phi / e } with c the box centre and
 * e = (n-1) h / 2.  grad (or NULL) receives [count][3] the analytic gradient d phi / d q of the same
 * interpolant at the clamped point (the cell's corner differences along each axis, interpolated
 * over the other two), which is also d(phi/e) / d x_hat. */
void or_nsdf_targets2(int32_t n, const float* origin, float spacing, const float* values, int64_t count,
                      const float* pts, double* rec, double* grad) {
  const double h = spacing, ext = (double)(n - 1) * h, e = 0.5 * ext;
  for (int64_t k = 0; k < count; ++k) {
    double q[3], t[3];
    int64_t i[3];
    for (int d = 0; d < 3; ++d) {
      const double lo = origin[d], hi = (double)origin[d] + ext;
      double v = pts[3 * k + d];
      v = v < lo ? lo : (v > hi ? hi : v);
      q[d] = v;
      const double u = (v - lo) / h;
      int64_t ii = (int64_t)floor(u);
      if (ii > n - 2) ii = n - 2;
      if (ii < 0) ii = 0;
      i[d] = ii;
      t[d] = u - (double)ii;
    }
    double phi = 0, gr[3] = {0, 0, 0};
    for (int c = 0; c < 8; ++c) {
      const int bit[3] = {c & 1, (c >> 1) & 1, c >> 2};
      double wt[3];
      for (int d = 0; d < 3; ++d) wt[d] = bit[d] ? t[d] : 1 - t[d];
      const double v = values[((i[2] + bit[2]) * n + (i[1] + bit[1])) * n + (i[0] + bit[0])];
      phi += wt[0] * wt[1] * wt[2] * v;
      for (int d = 0; d < 3; ++d) {
        /* d wt[d] / d q_d = +-1/h; the other two factors stay */
        const double others = wt[(d + 1) % 3] * wt[(d + 2) % 3];
        gr[d] += (bit[d] ? 1.0 : -1.0) / h * others * v;
      }
    }
    for (int d = 0; d < 3; ++d) rec[4 * k + d] = (q[d] - ((double)origin[d] + e)) / e;
    rec[4 * k + 3] = phi / e;
    if (grad)
      for (int d = 0; d < 3; ++d) grad[3 * k + d] = gr[d];
  }
}

void or_nsdf_targets(int32_t n, const float* origin, float spacing, const float* values, int64_t count,
                     const float* pts, double* rec) {
  or_nsdf_targets2(n, origin, spacing, values, count, pts, rec, NULL);
}
