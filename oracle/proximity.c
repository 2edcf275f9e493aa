/* CPU oracle for the ProximityTaxel (App. A.6).  TEST INFRASTRUCTURE ONLY.
 *
 * A taxel responds to the tracked object's surface mass inside its sensing sphere.  The object
 * carries a surface point cloud p_hat_i in its own frame (sampled once, at scene reset); in the
 * world p_i = R_O p_hat_i + p_O.  For taxel j of link L (probe centre q_j = p_L + R_L x_j, axis
 * a_j = R_L n_j, sensing radius R_j):
 *   P_j = { i : |p_i - q_j| < R_j },   P_ij = R_j - |p_i - q_j|                (penetration)
 *   v_tax = v_L + w_L x (q_j - p_L),   v_p_i = v_O + w_O x (p_i - p_O)           (point velocities)
 *   v_t,ij = (v_p_i - v_tax) - a_j ((v_p_i - v_tax) . a_j)                      (normal part removed)
 *   rho_b = density / max(N_active_b, 1)                                        (density scale)
 *   f_j = k rho_b sum_i P_ij a_j + k_s rho_b sum_i P_ij v_t,ij
 *   tau_j = k rho_b sum_i P_ij ((p_i - q_j) x a_j)
 * and the channels are R_L^T f_j and R_L^T tau_j.  N_active_b is the number of tracked points in
 * env b: the object's cloud size, or 0 without an object (then every channel is 0).
 * Radius noise perturbs R_j before the query: R_j + rho (2u - 1), u from Philox4x32-10 with
 * counter (env, taxel, step, 9); a per-probe gain (optional) scales the accumulated sums.
 *
 * Every point is visited (brute force), in FP64, in the order of the equations above.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "oracle.h"

typedef struct {
  int32_t num_envs, num_links, num_taxels, num_objects;
  const int32_t* link_offset;   /* [L+1] taxels sorted by link */
  const float* taxel_pos;       /* [T][3] x_j, link frame */
  const float* taxel_normal;    /* [T][3] n_j, unit */
  const float* taxel_radius;    /* [T] sensing radius R_j */
  const int32_t* cloud_offset;  /* [num_objects + 1] */
  const float* cloud;           /* [N][3] object-frame surface points */
  double k, k_s, density;
  uint64_t seed;
  double radius_rho;            /* 0: no radius noise */
} or_prox_problem;

static double u01(uint32_t x) { return (double)(2u * (x >> 9) + 1u) * (1.0 / 16777216.0); }

static void quat_R(const double q[4], double R[3][3]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}
static void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* link_state [S][13][E*L] (px py pz qw qx qy qz vx vy vz wx wy wz), obj_id [S][E],
 * obj_state [S][13][E] or NULL (object static at the origin), gain [E][T] or NULL.
 * ft [S][6][E][T] (fx fy fz tx ty tz, link frame); mass [S][E][T] or NULL: sum_i P_ij;
 * count [S][E][T] or NULL: the number of points inside the sphere (a record for error bounds). */
void or_prox_run(const or_prox_problem* P, const float* link_state, const int32_t* obj_id, const float* obj_state,
                 int64_t step0, int32_t S, const float* gain, double* ft, double* mass, double* count, int threads) {
  const int E = P->num_envs, L = P->num_links, T = P->num_taxels;
  const int64_t ET = (int64_t)E * T, EL = (int64_t)E * L;
  const uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
#pragma omp parallel for num_threads(threads) schedule(dynamic) collapse(2)
  for (int s = 0; s < S; ++s)
    for (int e = 0; e < E; ++e) {
      const int oid = obj_id[(int64_t)s * E + e];
      const int has = oid >= 0 && oid < P->num_objects;
      const int64_t n0 = has ? P->cloud_offset[oid] : 0, n1 = has ? P->cloud_offset[oid + 1] : 0;
      const double rho = P->density / (double)(n1 - n0 > 1 ? n1 - n0 : 1);
      double RO[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, pO[3] = {0, 0, 0}, vO[3] = {0, 0, 0}, wO[3] = {0, 0, 0};
      if (obj_state) {
        double v[13];
        for (int c = 0; c < 13; ++c) v[c] = obj_state[((int64_t)s * 13 + c) * E + e];
        quat_R(v + 3, RO);
        for (int i = 0; i < 3; ++i) {
          pO[i] = v[i];
          vO[i] = v[7 + i];
          wO[i] = v[10 + i];
        }
      }
      for (int l = 0; l < L; ++l) {
        double v[13];
        for (int c = 0; c < 13; ++c) v[c] = link_state[((int64_t)s * 13 + c) * EL + (int64_t)e * L + l];
        double RL[3][3], pL[3], vL[3], wL[3];
        quat_R(v + 3, RL);
        for (int i = 0; i < 3; ++i) {
          pL[i] = v[i];
          vL[i] = v[7 + i];
          wL[i] = v[10 + i];
        }
        for (int j = P->link_offset[l]; j < P->link_offset[l + 1]; ++j) {
          double q[3], a[3];
          for (int r = 0; r < 3; ++r) {
            q[r] = pL[r];
            a[r] = 0;
            for (int c = 0; c < 3; ++c) {
              q[r] += RL[r][c] * (double)P->taxel_pos[3 * j + c];
              a[r] += RL[r][c] * (double)P->taxel_normal[3 * j + c];
            }
          }
          double Rj = P->taxel_radius[j];
          if (P->radius_rho > 0) {
            const uint32_t ctr[4] = {(uint32_t)e, (uint32_t)j, (uint32_t)(step0 + s), 9u};
            uint32_t x[4];
            or_philox4x32_10(ctr, key, x);
            Rj += P->radius_rho * (2.0 * u01(x[0]) - 1.0);
            if (Rj < 0) Rj = 0;
          }
          double qL[3], vtax[3];
          for (int i = 0; i < 3; ++i) qL[i] = q[i] - pL[i];
          cross(wL, qL, vtax);
          for (int i = 0; i < 3; ++i) vtax[i] += vL[i];
          double f[3] = {0, 0, 0}, tau[3] = {0, 0, 0}, msum = 0, cnt = 0;
          for (int64_t i = n0; i < n1; ++i) {
            double p[3];
            for (int r = 0; r < 3; ++r) {
              p[r] = pO[r];
              for (int c = 0; c < 3; ++c) p[r] += RO[r][c] * (double)P->cloud[3 * i + c];
            }
            const double d = sqrt((p[0] - q[0]) * (p[0] - q[0]) + (p[1] - q[1]) * (p[1] - q[1]) +
                                  (p[2] - q[2]) * (p[2] - q[2]));
            if (!(d < Rj)) continue;
            const double Pij = Rj - d;
            double rO[3], vp[3], dv[3], vt[3], r[3], rxa[3];
            for (int c = 0; c < 3; ++c) rO[c] = p[c] - pO[c];
            cross(wO, rO, vp);
            for (int c = 0; c < 3; ++c) {
              vp[c] += vO[c];
              dv[c] = vp[c] - vtax[c];
            }
            const double dn = dv[0] * a[0] + dv[1] * a[1] + dv[2] * a[2];
            for (int c = 0; c < 3; ++c) {
              vt[c] = dv[c] - a[c] * dn;
              r[c] = p[c] - q[c];
            }
            cross(r, a, rxa);
            for (int c = 0; c < 3; ++c) {
              f[c] += P->k * rho * Pij * a[c] + P->k_s * rho * Pij * vt[c];
              tau[c] += P->k * rho * Pij * rxa[c];
            }
            msum += Pij;
            cnt += 1;
          }
          const double gj = gain ? (double)gain[(int64_t)e * T + j] : 1.0;
          for (int r = 0; r < 3; ++r) {   /* link frame: R_L^T f, R_L^T tau */
            double fl = 0, tl = 0;
            for (int c = 0; c < 3; ++c) {
              fl += RL[c][r] * f[c];
              tl += RL[c][r] * tau[c];
            }
            const int64_t k = (int64_t)e * T + j;
            ft[((int64_t)s * 6 + r) * ET + k] = gj * fl;
            ft[((int64_t)s * 6 + 3 + r) * ET + k] = gj * tl;
          }
          if (mass) mass[(int64_t)s * ET + (int64_t)e * T + j] = msum;
          if (count) count[(int64_t)s * ET + (int64_t)e * T + j] = cnt;
        }
      }
    }
}
