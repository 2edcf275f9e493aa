/* Driver for the sanitizer build of the CPU oracle (test infrastructure): a small scene with
 * every noise knob on, both precisions, a reset, the neural-SDF forward/gradient/Adam/targets and
 * the thermal solver.  Built with -fsanitize=address,undefined by tests/test_oracle_sanitize.py;
 * any out-of-bounds access, leak or undefined operation aborts the run. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

double or_nsdf_loss_grad(const double* P, int64_t n, const double* x, const double* target, double* grad, int bf16,
                         double pair_lambda);
void or_nsdf_adam(double* P, double* m, double* v, const double* g, int64_t np, int t, double lr, double b1, double b2,
                  double eps);
void or_nsdf_targets(int32_t n, const float* origin, float spacing, const float* values, int64_t count,
                     const float* pts, double* rec);

enum { E = 3, L = 3, T = 13, S = 4, N = 12, NP = 15681 };

static double urand(unsigned* s) {
  *s = *s * 1664525u + 1013904223u;
  return (double)(*s >> 8) / 16777216.0;
}

int main(void) {
  unsigned seed = 12345u;
  int32_t off[L + 1] = {0, 5, 5, T};   /* an empty middle link */
  float pos[T * 3], nrm[T * 3], rad[T];
  for (int j = 0; j < T; ++j) {
    pos[3 * j] = 0.002f * (float)(j % 4);
    pos[3 * j + 1] = 0.002f * (float)(j / 4);
    pos[3 * j + 2] = 0.f;
    nrm[3 * j] = 0.f; nrm[3 * j + 1] = 0.f; nrm[3 * j + 2] = 1.f;
    rad[j] = j == 7 ? 0.f : 1e-3f;     /* one inactive filler */
  }
  float vals[N * N * N];
  const float h = 0.1f / (N - 1), o = -0.05f;
  for (int z = 0; z < N; ++z)
    for (int y = 0; y < N; ++y)
      for (int x = 0; x < N; ++x) {
        const float px = o + h * x, py = o + h * y, pz = o + h * z;
        vals[(z * N + y) * N + x] = sqrtf(px * px + py * py + pz * pz) - 0.03f;
      }
  or_grid g[2];
  memset(g, 0, sizeof(g));
  for (int k = 0; k < 2; ++k) {
    g[k].n = N; g[k].origin[0] = g[k].origin[1] = g[k].origin[2] = o; g[k].spacing = h; g[k].values = vals;
  }
  double* nsdf = calloc((size_t)2 * NP, sizeof(double));
  for (int i = 0; i < 2 * NP; ++i) nsdf[i] = 0.2 * (urand(&seed) - 0.5);
  or_problem P;
  memset(&P, 0, sizeof(P));
  P.num_envs = E; P.num_links = L; P.num_taxels = T; P.num_objects = 2;
  P.link_offset = off; P.taxel_pos = pos; P.taxel_normal = nrm; P.taxel_radius = rad; P.grids = g;
  P.k_n = 500.f; P.c_n = 1.f; P.alpha = 1.2f; P.k_t = 2.f; P.k_w = 2.f; P.mu = 0.8f; P.prox_range = 0.01f;
  P.eta_on = 5e-4f; P.noise_on = 1; P.seed = 99; P.drift_sigma = 1e-3f; P.white_sigma = 2e-3f; P.bias = 0.01f;
  P.quant_step = 0.01f; P.hyst_mode = 1; P.tau_load = 2.f; P.tau_unload = 6.f; P.maxwell_beta = 0.5f;
  P.maxwell_tau = 0.05f; P.dt = 0.005f; P.p_dead = 0.2f; P.stuck_lo = 0.1f; P.stuck_hi = 0.2f;
  P.radius_rho = 3e-4f; P.gain_lo = 0.9f; P.gain_hi = 1.1f; P.xtalk_kind = 2; P.xtalk_chi = 0.1f;
  P.xtalk_sigma = 2e-3f; P.eta_off = 2e-4f; P.nsdf_band = 1e-3f; P.nsdf_params = nsdf;

  float ls[S * 13 * E * L], os[S * 13 * E];
  int32_t oid[S * E];
  for (int s = 0; s < S; ++s) {
    for (int c = 0; c < 13; ++c)
      for (int i = 0; i < E * L; ++i) ls[(s * 13 + c) * E * L + i] = (float)(0.04 * (urand(&seed) - 0.5));
    for (int i = 0; i < E * L; ++i) {   /* unit quaternions */
      float* q = &ls[(s * 13 + 3) * E * L + i];
      double w = urand(&seed) - 0.5, x = urand(&seed) - 0.5, y = urand(&seed) - 0.5, z = urand(&seed) - 0.5;
      double nn = sqrt(w * w + x * x + y * y + z * z);
      q[0] = (float)(w / nn); q[E * L] = (float)(x / nn); q[2 * E * L] = (float)(y / nn); q[3 * E * L] = (float)(z / nn);
    }
    for (int c = 0; c < 13; ++c)
      for (int e = 0; e < E; ++e) os[(s * 13 + c) * E + e] = c == 3 ? 1.f : (c >= 7 ? 0.1f : 0.f);
    for (int e = 0; e < E; ++e) oid[s * E + e] = e == 2 ? -1 : e;
  }
  const size_t ET = (size_t)E * T, EL = (size_t)E * L;
  or_state st;
  st.drift = calloc(6 * ET, 8); st.hyst = calloc(6 * ET, 8); st.hyst_prev = calloc(6 * ET, 8);
  st.schmitt = calloc(ET, 1); st.dead = calloc(ET, 1); st.stuck = calloc(ET, 8); st.gain = calloc(ET, 8);
  or_outputs out;
  out.bit = calloc(S * ET, 1); out.bit_noisy = calloc(S * ET, 1);
  out.depth = calloc(S * ET, 8); out.prox = calloc(S * ET, 8); out.surfdist = calloc(S * ET, 8);
  out.ft = calloc(S * 6 * ET, 8); out.ft_noisy = calloc(S * 6 * ET, 8); out.normal = calloc(S * 3 * ET, 8);
  out.link_sums = calloc(S * 11 * EL, 8); out.link_sums_noisy = calloc(S * 11 * EL, 8);
  out.xtalk_scale = calloc(S * 6 * ET, 8);
  or_inputs in = {ls, oid, os, 5, S};
  double check = 0;
  for (int mode = 0; mode < 4; ++mode) {
    P.hyst_mode = mode == 3 ? 2 : 1;
    P.xtalk_kind = mode == 1 ? 1 : 2;
    P.sdf_mode = mode == 2 ? 1 : 0;
    if (or_reset_f32(&P, &st, NULL, 3) || or_run_f32(&P, &in, &out, &st, 1)) return 2;
    for (size_t i = 0; i < S * 6 * ET; ++i) check += out.ft_noisy[i];
    if (or_reset_f64(&P, &st, NULL, 3) || or_run_f64(&P, &in, &out, &st, 1)) return 3;
    for (size_t i = 0; i < S * 11 * EL; ++i) check += out.link_sums_noisy[i];
  }
  /* neural surrogate: loss gradient (plain and paired), Adam, targets */
  enum { NS = 8 };
  double xs[NS * 3], tg[NS], gr[NP], m[NP], v[NP], rec[NS * 4];
  float pts[NS * 3];
  for (int i = 0; i < NS * 3; ++i) { xs[i] = 2 * urand(&seed) - 1; pts[i] = (float)(0.06 * (urand(&seed) - 0.5)); }
  for (int i = 0; i < NS; ++i) tg[i] = urand(&seed) - 0.5;
  memset(m, 0, sizeof(m)); memset(v, 0, sizeof(v));
  check += or_nsdf_loss_grad(nsdf, NS, xs, tg, gr, 1, 0.0);
  check += or_nsdf_loss_grad(nsdf, NS, xs, tg, gr, 0, 1.0);
  or_nsdf_adam(nsdf, m, v, gr, NP, 1, 1e-3, 0.9, 0.999, 1e-8);
  or_nsdf_targets(N, g[0].origin, h, vals, NS, pts, rec);
  for (int i = 0; i < NS * 4; ++i) check += rec[i];
  /* thermal fields on link 0 and 2 */
  int32_t fl[2] = {0, 2};
  float tobj[E] = {30.f, 40.f, 50.f};
  or_thermal th = {2, fl, 16, 1e-3f, {-8e-3f, -8e-3f, -16e-3f}, 1e-3f, 0.2f, 2e6f, 0.85f, 10.f, 1.f, 22.f, 22.f,
                   0.1f, tobj};
  float* f32 = malloc(sizeof(float) * E * 2 * 4096);
  double* f64 = malloc(sizeof(double) * E * 2 * 4096);
  for (int i = 0; i < E * 2 * 4096; ++i) { f32[i] = 22.f; f64[i] = 22.0; }
  double* tt = calloc(S * ET, 8);
  double* led = calloc(S * E * 2 * 2, 8);
  or_thermal_run_f32(&th, E, T, off, pos, out.depth, S, f32, tt, led);
  or_thermal_run_f64(&th, E, T, off, pos, out.depth, S, f64, tt, led);
  check += f32[100] + f64[200] + tt[3];
  printf("sanitized oracle run ok %.6g\n", check);
  free(f32); free(f64); free(tt); free(led); free(nsdf);
  free(st.drift); free(st.hyst); free(st.hyst_prev); free(st.schmitt); free(st.dead); free(st.stuck); free(st.gain);
  free(out.bit); free(out.bit_noisy); free(out.depth); free(out.prox); free(out.surfdist); free(out.ft);
  free(out.ft_noisy); free(out.normal); free(out.link_sums); free(out.link_sums_noisy); free(out.xtalk_scale);
  return 0;
}
