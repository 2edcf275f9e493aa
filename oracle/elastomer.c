/* CPU oracle for the ElastomerTaxel (App. A.7).  TEST INFRASTRUCTURE ONLY.
 *
 * Marker displacements of a deformable pad from SDF-driven dilation and anchored shear history.
 * For a sensor link with markers j (link-frame positions x_j, unit normals n_j) and the tangent
 * projection Pi_n(z) = z - (z . n) n:
 *   dilation, source probe i of the same link with penetration h_i:
 *     r_ij = Pi_{n_j}(x_j - x_i),  g = exp(-lambda_d |r|^2),  rho = 1 / (|r|^2 + eps^2)
 *     w_ij = h_i (c g / g_bar + (1 - c) rho / rho_bar),  g_bar = e^{-1/2} / sqrt(2 lambda_d),
 *            rho_bar = 1 / (2 eps)
 *     u^d_ij = s_d (r_ij w_ij + n_j h_i^alpha g(r_ij))
 *   shear, tracked surface point p of the env's object (sensor-frame position z_p, anchor e_p,
 *   penetration h_p into the pad):
 *     u^s_pj = s_s Pi_{n_j}(z_p - e_p) h_p exp(-lambda_s |Pi_{n_j}(x_j - z_p)|^2)
 *   y_j = sum_i u^d_ij + sum_p u^s_pj.
 * Anchors: a point without an anchor takes e_p = z_p when the pad's SDF at z_p drops below
 * -eta_enter; an anchored point drops its anchor when the SDF rises above +eta_exit.
 *
 * Readings (where the paper leaves the form open):
 *   - the source probes are the readout's own probes on the sensor link; their penetration
 *     h_i = max(0, -phi(q_i)) is read from the readout's depth d_i = max(0, R_i - phi(q_i)) as
 *     max(0, d_i - R_i) (FP32, as the kernel forms it);
 *   - the pad is a box in the link frame (centre and half extents given per sensor link); its
 *     SDF is the exact box distance, and h_p = max(0, -SDF);
 *   - the tracked points are one surface cloud per object, object frame, posed by the object's
 *     state each step: z_p = R_L^T (R_O p_hat + p_O - p_L);
 *   - anchors belong to (env, sensor link, point index); a change of the env's object clears them.
 *
 * The point positions, the pad SDF and the anchor decisions follow one written FP32 sequence
 * (contraction off, fused multiply-adds written as fmaf), so that the decisions, which are
 * comparisons, are the same on any IEEE machine; the sums are FP64 from those values.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t num_envs, num_links, num_taxels, num_objects;
  const int32_t* link_offset;   /* [L+1] */
  const float* taxel_pos;       /* [T][3] */
  const float* taxel_normal;    /* [T][3] */
  const float* taxel_radius;    /* [T] the readout's probe radius R_j */
  int32_t num_sensor_links;
  const int32_t* sensor_links;  /* [Ls] */
  const float* pad_center;      /* [Ls][3] link frame */
  const float* pad_half;        /* [Ls][3] half extents */
  const int32_t* cloud_offset;  /* [num_objects + 1] */
  const float* cloud;           /* [N][3] object frame */
  double s_d, s_s, lambda_d, lambda_s, alpha, c, eps;
  float eta_enter, eta_exit;
  int32_t max_points;           /* anchor slots per (env, sensor link) */
} or_elast_problem;

typedef struct {
  float* anchor;       /* [E][Ls][max_points][3] */
  uint8_t* active;     /* [E][Ls][max_points] */
  int32_t* last_oid;   /* [E][Ls]; -2 before the first step */
} or_elast_state;

/* ---- the FP32 sequence: pose, point position, pad SDF ---- */
static void quat_R32(float w, float x, float y, float z, float R[9]) {
  const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  R[0] = 1.0f - 2.0f * (yy + zz);
  R[1] = 2.0f * (xy - wz);
  R[2] = 2.0f * (xz + wy);
  R[3] = 2.0f * (xy + wz);
  R[4] = 1.0f - 2.0f * (xx + zz);
  R[5] = 2.0f * (yz - wx);
  R[6] = 2.0f * (xz - wy);
  R[7] = 2.0f * (yz + wx);
  R[8] = 1.0f - 2.0f * (xx + yy);
}
static void mv32(const float R[9], float x0, float x1, float x2, float y[3]) {
  for (int i = 0; i < 3; ++i) y[i] = fmaf(R[3 * i + 2], x2, fmaf(R[3 * i + 1], x1, R[3 * i] * x0));
}
static void mtv32(const float R[9], float x0, float x1, float x2, float y[3]) {
  for (int i = 0; i < 3; ++i) y[i] = fmaf(R[6 + i], x2, fmaf(R[3 + i], x1, R[i] * x0));
}
/* exact SDF of the box |z - ctr| <= half */
static float box_sdf32(const float z[3], const float ctr[3], const float half[3]) {
  float q[3], m[3];
  for (int k = 0; k < 3; ++k) {
    q[k] = fabsf(z[k] - ctr[k]) - half[k];
    m[k] = fmaxf(q[k], 0.0f);
  }
  const float out = sqrtf(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
  const float in = fminf(fmaxf(q[0], fmaxf(q[1], q[2])), 0.0f);
  return out + in;
}

/* ---- FP64 terms ---- */
static void tproj(const double v[3], const double n[3], double out[3]) {
  const double d = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
  for (int k = 0; k < 3; ++k) out[k] = v[k] - d * n[k];
}

void or_elast_state_clear(const or_elast_problem* P, or_elast_state* st) {
  const int64_t n = (int64_t)P->num_envs * P->num_sensor_links;
  memset(st->anchor, 0, (size_t)(n * P->max_points * 3) * sizeof(float));
  memset(st->active, 0, (size_t)(n * P->max_points));
  for (int64_t i = 0; i < n; ++i) st->last_oid[i] = -2;
}

/* link_state [S][13][E*L], obj_id [S][E], obj_state [S][13][E] or NULL, depth [S][E][T] (the
 * readout's clean depth).  disp [S][3][E][T] and absum [S][E][T] (sum of |u| over the terms, for
 * error bounds) are written for the sensor links' markers only. */
void or_elast_run(const or_elast_problem* P, or_elast_state* st, const float* link_state, const int32_t* obj_id,
                  const float* obj_state, const float* depth, int32_t S, double* disp, double* absum, int threads) {
  const int E = P->num_envs, L = P->num_links, T = P->num_taxels, Ls = P->num_sensor_links, NP = P->max_points;
  const int64_t EL = (int64_t)E * L, ET = (int64_t)E * T;
  const double gbar = exp(-0.5) / sqrt(2.0 * P->lambda_d), rbar = 1.0 / (2.0 * P->eps);
#pragma omp parallel for num_threads(threads) schedule(dynamic)
  for (int e = 0; e < E; ++e) {
    float* z = (float*)malloc((size_t)(NP > 0 ? NP : 1) * 3 * sizeof(float));
    float* hp = (float*)malloc((size_t)(NP > 0 ? NP : 1) * sizeof(float));
    for (int s = 0; s < S; ++s) {
      const int oid = obj_id[(int64_t)s * E + e];
      const int has = oid >= 0 && oid < P->num_objects;
      float RO[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, pO[3] = {0, 0, 0};
      if (has && obj_state) {
        float v[13];
        for (int c = 0; c < 13; ++c) v[c] = obj_state[((int64_t)s * 13 + c) * E + e];
        quat_R32(v[3], v[4], v[5], v[6], RO);
        for (int k = 0; k < 3; ++k) pO[k] = v[k];
      }
      const int n0 = has ? P->cloud_offset[oid] : 0, n1 = has ? P->cloud_offset[oid + 1] : 0;
      for (int li = 0; li < Ls; ++li) {
        const int l = P->sensor_links[li];
        const int64_t sl = (int64_t)e * Ls + li;
        float* anc = st->anchor + sl * NP * 3;
        uint8_t* act = st->active + sl * NP;
        if (st->last_oid[sl] != oid) {   /* a change of object clears the anchors */
          memset(anc, 0, (size_t)NP * 3 * sizeof(float));
          memset(act, 0, (size_t)NP);
          st->last_oid[sl] = oid;
        }
        float v[13];
        for (int c = 0; c < 13; ++c) v[c] = link_state[((int64_t)s * 13 + c) * EL + (int64_t)e * L + l];
        float RL[9];
        quat_R32(v[3], v[4], v[5], v[6], RL);
        /* tracked points: position in the sensor frame, pad SDF, anchor update */
        const int np = n1 - n0;
        for (int k = 0; k < np; ++k) {
          const float* ph = P->cloud + 3 * (int64_t)(n0 + k);
          float w[3], d[3];
          mv32(RO, ph[0], ph[1], ph[2], w);
          for (int q = 0; q < 3; ++q) d[q] = (w[q] + pO[q]) - v[q];
          mtv32(RL, d[0], d[1], d[2], z + 3 * k);
          const float phi = box_sdf32(z + 3 * k, P->pad_center + 3 * li, P->pad_half + 3 * li);
          if (!act[k] && phi < -P->eta_enter) {
            act[k] = 1;
            for (int q = 0; q < 3; ++q) anc[3 * k + q] = z[3 * k + q];
          } else if (act[k] && phi > P->eta_exit) {
            act[k] = 0;
          }
          hp[k] = fmaxf(-phi, 0.0f);
        }
        /* marker displacements */
        const int j0 = P->link_offset[l], j1 = P->link_offset[l + 1];
        for (int j = j0; j < j1; ++j) {
          double xj[3], nj[3], y[3] = {0, 0, 0}, a = 0;
          for (int q = 0; q < 3; ++q) {
            xj[q] = P->taxel_pos[3 * j + q];
            nj[q] = P->taxel_normal[3 * j + q];
          }
          for (int i = j0; i < j1; ++i) {   /* dilation */
            const float hf = fmaxf(depth[(int64_t)s * ET + (int64_t)e * T + i] - P->taxel_radius[i], 0.0f);
            if (!(hf > 0.0f)) continue;
            const double h = hf;
            double dx[3], r[3];
            for (int q = 0; q < 3; ++q) dx[q] = xj[q] - (double)P->taxel_pos[3 * i + q];
            tproj(dx, nj, r);
            const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const double g = exp(-P->lambda_d * r2);
            const double rho = 1.0 / (r2 + P->eps * P->eps);
            const double wij = h * (P->c * g / gbar + (1.0 - P->c) * rho / rbar);
            const double ha = pow(h, P->alpha);
            double u[3];
            for (int q = 0; q < 3; ++q) u[q] = P->s_d * (r[q] * wij + nj[q] * ha * g);
            for (int q = 0; q < 3; ++q) y[q] += u[q];
            a += sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
          }
          for (int k = 0; k < np; ++k) {    /* shear */
            if (!act[k] || !(hp[k] > 0.0f)) continue;
            double ze[3], xz[3], t1[3], t2[3];
            for (int q = 0; q < 3; ++q) {
              ze[q] = (double)z[3 * k + q] - (double)anc[3 * k + q];
              xz[q] = xj[q] - (double)z[3 * k + q];
            }
            tproj(ze, nj, t1);
            tproj(xz, nj, t2);
            const double t22 = t2[0] * t2[0] + t2[1] * t2[1] + t2[2] * t2[2];
            const double f = P->s_s * (double)hp[k] * exp(-P->lambda_s * t22);
            double u[3];
            for (int q = 0; q < 3; ++q) u[q] = f * t1[q];
            for (int q = 0; q < 3; ++q) y[q] += u[q];
            a += sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
          }
          for (int q = 0; q < 3; ++q) disp[((int64_t)s * 3 + q) * ET + (int64_t)e * T + j] = y[q];
          if (absum) absum[(int64_t)s * ET + (int64_t)e * T + j] = a;
        }
      }
    }
    free(z);
    free(hp);
  }
}
