/* Driver for the sanitizer build of the sensor oracles (test infrastructure): one of the
 * ProximityTaxel, ElastomerTaxel or raycast oracles, chosen at compile time (SAN_PROX, SAN_ELAST,
 * SAN_RAY), runs a small scene: three envs, one of them without an object and one with an object
 * id out of range, an empty link, a probe of radius 0, a few steps with moving poses.  Built with
 * -fsanitize=address,undefined by tests/test_oracle_sanitize.py; any out-of-bounds access, leak or
 * undefined operation aborts the run. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#if defined(SAN_PROX)
#include "../oracle/proximity.c"
#elif defined(SAN_ELAST)
#include "../oracle/elastomer.c"
#elif defined(SAN_RAY)
#include "../oracle/raycast.c"
#else
#error "choose SAN_PROX, SAN_ELAST or SAN_RAY"
#endif

enum { E = 3, L = 3, T = 13, S = 4, NPTS = 200 };

static double urand(unsigned* s) {
  *s = *s * 1664525u + 1013904223u;
  return (double)(*s >> 8) / 16777216.0;
}

int main(void) {
  unsigned seed = 777u;
  int32_t off[L + 1] = {0, 6, 6, T};   /* an empty middle link */
  float pos[T * 3], nrm[T * 3], rad[T];
  for (int j = 0; j < T; ++j) {
    pos[3 * j] = 0.002f * (float)(j % 4) - 0.003f;
    pos[3 * j + 1] = 0.002f * (float)(j / 4) - 0.003f;
    pos[3 * j + 2] = 0.f;
    nrm[3 * j] = 0.f; nrm[3 * j + 1] = 0.f; nrm[3 * j + 2] = 1.f;
    rad[j] = j == 4 ? 0.f : 2e-3f;
  }
  /* link poses: near the object centre, small rotations; link_state [S][13][E*L] */
  float* ls = calloc((size_t)S * 13 * E * L, sizeof(float));
  for (int s = 0; s < S; ++s)
    for (int i = 0; i < E * L; ++i) {
      float* c = ls + (size_t)s * 13 * E * L + i;
      const size_t st = (size_t)E * L;
      c[0] = (float)(0.004 * (urand(&seed) - 0.5));
      c[st] = (float)(0.004 * (urand(&seed) - 0.5));
      c[2 * st] = (float)(0.012 + 0.006 * (urand(&seed) - 0.5));
      double q[4] = {1.0, 0.1 * (urand(&seed) - 0.5), 0.1 * (urand(&seed) - 0.5), 0.1 * (urand(&seed) - 0.5)};
      const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
      for (int k = 0; k < 4; ++k) c[(3 + k) * st] = (float)(q[k] / nq);
      for (int k = 7; k < 13; ++k) c[k * st] = (float)(0.01 * (urand(&seed) - 0.5));
    }
  int32_t oid[S * E];
  for (int s = 0; s < S; ++s) { oid[s * E] = 0; oid[s * E + 1] = -1; oid[s * E + 2] = s == 2 ? 5 : 0; }
  double check = 0.0;
#if defined(SAN_PROX) || defined(SAN_ELAST)
  /* one object: points on a sphere of radius 1.2 cm */
  int32_t coff[2] = {0, NPTS};
  float cloud[NPTS * 3];
  for (int i = 0; i < NPTS; ++i) {
    const double z = 2.0 * urand(&seed) - 1.0, ph = 6.283185307179586 * urand(&seed), r = sqrt(1.0 - z * z);
    cloud[3 * i] = (float)(0.012 * r * cos(ph));
    cloud[3 * i + 1] = (float)(0.012 * r * sin(ph));
    cloud[3 * i + 2] = (float)(0.012 * z);
  }
#endif
#if defined(SAN_PROX)
  or_prox_problem P = {E, L, T, 1, off, pos, nrm, rad, coff, cloud, 50.0, 5.0, 1.0, 0x1234ull, 2e-4};
  double* ft = calloc((size_t)S * 6 * E * T, sizeof(double));
  double* mass = calloc((size_t)S * E * T, sizeof(double));
  double* cnt = calloc((size_t)S * E * T, sizeof(double));
  or_prox_run(&P, ls, oid, NULL, 3, S, NULL, ft, mass, cnt, 1);
  for (size_t i = 0; i < (size_t)S * 6 * E * T; ++i) check += ft[i];
  free(ft); free(mass); free(cnt);
#elif defined(SAN_ELAST)
  int32_t sl[2] = {0, 2};
  float pc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, ph[6] = {0.004f, 0.004f, 0.001f, 0.004f, 0.004f, 0.001f};
  or_elast_problem P = {E, L, T, 1, off, pos, nrm, rad, 2, sl, pc, ph, coff, cloud,
                        1.0, 0.5, 2e-6, 2e-6, 1.0, 1.0, 1e-4, 2e-3f, 4e-3f, NPTS};
  or_elast_state st;
  st.anchor = calloc((size_t)E * 2 * NPTS * 3, sizeof(float));
  st.active = calloc((size_t)E * 2 * NPTS, 1);
  st.last_oid = calloc((size_t)E * 2, sizeof(int32_t));
  or_elast_state_clear(&P, &st);
  float* depth = calloc((size_t)S * E * T, sizeof(float));
  for (size_t i = 0; i < (size_t)S * E * T; ++i) depth[i] = (float)(3e-3 * urand(&seed));
  double* disp = calloc((size_t)S * 3 * E * T, sizeof(double));
  double* absum = calloc((size_t)S * E * T, sizeof(double));
  or_elast_run(&P, &st, ls, oid, NULL, depth, S, disp, absum, 1);
  or_elast_run(&P, &st, ls, oid, NULL, depth, S, disp, absum, 1);   /* anchors carried over */
  for (size_t i = 0; i < (size_t)S * 3 * E * T; ++i) check += disp[i];
  free(st.anchor); free(st.active); free(st.last_oid); free(depth); free(disp); free(absum);
#elif defined(SAN_RAY)
  /* one object: a closed cube of half-edge 1 cm, outward faces */
  const float a = 0.01f;
  float verts[8 * 3];
  for (int i = 0; i < 8; ++i) {
    verts[3 * i] = (i & 1) ? a : -a;
    verts[3 * i + 1] = (i & 2) ? a : -a;
    verts[3 * i + 2] = (i & 4) ? a : -a;
  }
  int32_t tris[12 * 3] = {0, 2, 1, 1, 2, 3, 4, 5, 6, 5, 7, 6, 0, 1, 4, 1, 5, 4,
                          2, 6, 3, 3, 6, 7, 0, 4, 2, 2, 4, 6, 1, 3, 5, 3, 7, 5};
  int32_t voff[2] = {0, 8}, toff[2] = {0, 12};
  or_ray_problem P = {E, L, T, 1, off, pos, nrm, rad, voff, verts, toff, tris};
  double* depth = calloc((size_t)S * E * T, sizeof(double));
  double* normal = calloc((size_t)S * 3 * E * T, sizeof(double));
  int32_t* tri = calloc((size_t)S * E * T, sizeof(int32_t));
  int32_t* tq = calloc((size_t)S * E * T, sizeof(int32_t));
  double* tp = calloc((size_t)S * E * T, sizeof(double));
  for (size_t i = 0; i < (size_t)S * E * T; ++i) tq[i] = (int32_t)(i % 13) - 1;   /* -1 .. 11 */
  or_ray_run(&P, ls, oid, NULL, S, depth, normal, tri, tq, tp, 1);
  for (size_t i = 0; i < (size_t)S * E * T; ++i) check += depth[i] + (double)tri[i];
  free(depth); free(normal); free(tri); free(tq); free(tp);
#endif
  free(ls);
  if (!isfinite(check)) return 4;
  printf("sanitized sensor oracle run ok %.6g\n", check);
  return 0;
}
