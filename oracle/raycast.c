/* CPU oracle for the raycast contact-depth backend (App. A.1).  TEST INFRASTRUCTURE ONLY.
 *
 * Probe j of link L: centre q_j = p_L + R_L x_j, axis a_j = R_L n_j (pointing toward the
 * object), radius R_j.  The object is a closed triangle mesh with outward faces, in its own frame
 * (posed by p_O, R_O).  For each triangle:
 *   - sphere test: the closest point of the triangle to q_j at distance dist gives a penetration
 *     R_j - dist;
 *   - ray test: a ray from q_j along -a_j (away from the object); if its first crossing with the
 *     mesh leaves the mesh (the face's outward normal has a positive component along the ray),
 *     q_j lies inside the object, t below that face along the axis, and the penetration is
 *     R_j + t, i.e. R_j minus the hit's signed distance along a_j.
 * The deepest penetration over the triangles and the two tests wins; the depth is its positive
 * part and the contact normal is the outward face normal of the winning triangle (link frame).
 * A probe with R_j = 0 reads zero.
 *
 * Every triangle is visited (no BVH), in FP64, in the order above: sphere tests in triangle
 * order, then the ray's first hit; a later candidate wins only if strictly deeper.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
  int32_t num_envs, num_links, num_taxels, num_objects;
  const int32_t* link_offset;   /* [L+1] */
  const float* taxel_pos;       /* [T][3] */
  const float* taxel_normal;    /* [T][3] */
  const float* taxel_radius;    /* [T] */
  const int32_t* vert_offset;   /* [num_objects + 1] */
  const float* verts;           /* [V][3] object frame */
  const int32_t* tri_offset;    /* [num_objects + 1] */
  const int32_t* tris;          /* [M][3] vertex indices within the object's vertices */
} or_ray_problem;

static void quatR(const double q[4], double R[3][3]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double* a, const double* b, double* c) {
  for (int i = 0; i < 3; ++i) c[i] = a[i] - b[i];
}
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* closest point of triangle (A, B, C) to P by the triangle's Voronoi regions: the vertex, edge or
 * face region that contains P's projection (the published method of Ericson, Real-Time Collision
 * Detection, sec. 5.1.5) */
static void closest_point(const double* P, const double* A, const double* B, const double* C, double* X) {
  double AB[3], AC[3], AP[3];
  sub3(B, A, AB); sub3(C, A, AC); sub3(P, A, AP);
  const double d1 = dot3(AB, AP), d2 = dot3(AC, AP);
  if (d1 <= 0 && d2 <= 0) { for (int i = 0; i < 3; ++i) X[i] = A[i]; return; }
  double BP[3];
  sub3(P, B, BP);
  const double d3 = dot3(AB, BP), d4 = dot3(AC, BP);
  if (d3 >= 0 && d4 <= d3) { for (int i = 0; i < 3; ++i) X[i] = B[i]; return; }
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0 && d1 >= 0 && d3 <= 0) {
    const double v = d1 / (d1 - d3);
    for (int i = 0; i < 3; ++i) X[i] = A[i] + v * AB[i];
    return;
  }
  double CP[3];
  sub3(P, C, CP);
  const double d5 = dot3(AB, CP), d6 = dot3(AC, CP);
  if (d6 >= 0 && d5 <= d6) { for (int i = 0; i < 3; ++i) X[i] = C[i]; return; }
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0 && d2 >= 0 && d6 <= 0) {
    const double w = d2 / (d2 - d6);
    for (int i = 0; i < 3; ++i) X[i] = A[i] + w * AC[i];
    return;
  }
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
    const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    for (int i = 0; i < 3; ++i) X[i] = B[i] + w * (C[i] - B[i]);
    return;
  }
  const double den = 1.0 / (va + vb + vc), v = vb * den, w = vc * den;
  for (int i = 0; i < 3; ++i) X[i] = A[i] + AB[i] * v + AC[i] * w;
}

/* ray O + t D against triangle (A, B, C): t > 0 and the barycentric coordinates in [0, 1]
 * (Moller-Trumbore); returns 0 for no hit */
static int ray_hit(const double* O, const double* D, const double* A, const double* B, const double* C, double* t) {
  double E1[3], E2[3], Pv[3], Tv[3], Qv[3];
  sub3(B, A, E1); sub3(C, A, E2);
  cross3(D, E2, Pv);
  const double det = dot3(E1, Pv);
  if (det == 0.0) return 0;
  const double inv = 1.0 / det;
  sub3(O, A, Tv);
  const double u = dot3(Tv, Pv) * inv;
  if (u < 0.0 || u > 1.0) return 0;
  cross3(Tv, E1, Qv);
  const double v = dot3(D, Qv) * inv;
  if (v < 0.0 || u + v > 1.0) return 0;
  const double tt = dot3(E2, Qv) * inv;
  if (!(tt > 0.0)) return 0;
  *t = tt;
  return 1;
}

static void face_normal(const double* A, const double* B, const double* C, double* n) {
  double E1[3], E2[3];
  sub3(B, A, E1); sub3(C, A, E2);
  cross3(E1, E2, n);
  const double l = sqrt(dot3(n, n));
  for (int i = 0; i < 3; ++i) n[i] /= l;
}

/* penetration of probe (q, a, R) against triangle k alone (both tests; the ray test counts the
 * hit only if it leaves the mesh), -inf when neither test applies */
static double tri_pen(const double* q, const double* a, double R, const double* A, const double* B, const double* C) {
  double X[3], d[3], nrm[3], D[3] = {-a[0], -a[1], -a[2]}, t;
  closest_point(q, A, B, C, X);
  sub3(q, X, d);
  double pen = R - sqrt(dot3(d, d));
  face_normal(A, B, C, nrm);
  if (ray_hit(q, D, A, B, C, &t) && dot3(D, nrm) > 0.0 && R + t > pen) pen = R + t;
  return pen;
}

/* link_state [S][13][E*L], obj_id [S][E], obj_state [S][13][E] or NULL.  Outputs: depth [S][E][T],
 * normal [S][3][E][T] (link frame, 0 without contact), tri [S][E][T] (winning triangle within its
 * object, -1 without contact).  tri_query [S][E][T] or NULL: for each probe the penetration of
 * that triangle alone goes to tri_pen [S][E][T] (-inf for -1). */
void or_ray_run(const or_ray_problem* P, const float* link_state, const int32_t* obj_id, const float* obj_state,
                int32_t S, double* depth, double* normal, int32_t* tri, const int32_t* tri_query, double* tri_pen_out,
                int threads) {
  const int E = P->num_envs, L = P->num_links, T = P->num_taxels;
  const int64_t EL = (int64_t)E * L, ET = (int64_t)E * T;
#pragma omp parallel for num_threads(threads) schedule(dynamic) collapse(2)
  for (int s = 0; s < S; ++s)
    for (int e = 0; e < E; ++e) {
      const int oid = obj_id[(int64_t)s * E + e];
      const int has = oid >= 0 && oid < P->num_objects;
      double RO[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, pO[3] = {0, 0, 0};
      if (has && obj_state) {
        double v[13];
        for (int c = 0; c < 13; ++c) v[c] = obj_state[((int64_t)s * 13 + c) * E + e];
        quatR(v + 3, RO);
        for (int i = 0; i < 3; ++i) pO[i] = v[i];
      }
      const float* V = has ? P->verts + 3 * (int64_t)P->vert_offset[oid] : P->verts;
      const int32_t* TR = has ? P->tris + 3 * (int64_t)P->tri_offset[oid] : P->tris;
      const int nt = has ? P->tri_offset[oid + 1] - P->tri_offset[oid] : 0;
      for (int l = 0; l < L; ++l) {
        double v[13], RL[3][3];
        for (int c = 0; c < 13; ++c) v[c] = link_state[((int64_t)s * 13 + c) * EL + (int64_t)e * L + l];
        quatR(v + 3, RL);
        for (int j = P->link_offset[l]; j < P->link_offset[l + 1]; ++j) {
          const int64_t k = (int64_t)e * T + j;
          const double R = P->taxel_radius[j];
          double qw[3], aw[3], q[3], a[3];
          for (int r = 0; r < 3; ++r) {
            qw[r] = v[r];
            aw[r] = 0;
            for (int c = 0; c < 3; ++c) {
              qw[r] += RL[r][c] * (double)P->taxel_pos[3 * j + c];
              aw[r] += RL[r][c] * (double)P->taxel_normal[3 * j + c];
            }
          }
          for (int r = 0; r < 3; ++r) {   /* object frame: R_O^T (q - p_O), R_O^T a */
            q[r] = 0;
            a[r] = 0;
            for (int c = 0; c < 3; ++c) {
              q[r] += RO[c][r] * (qw[c] - pO[c]);
              a[r] += RO[c][r] * aw[c];
            }
          }
          double best = 0.0;
          int bt = -1;
          if (R > 0) {
            for (int t = 0; t < nt; ++t) {   /* sphere tests */
              double A[3], B[3], C[3], X[3], d[3];
              for (int i = 0; i < 3; ++i) {
                A[i] = V[3 * TR[3 * t] + i]; B[i] = V[3 * TR[3 * t + 1] + i]; C[i] = V[3 * TR[3 * t + 2] + i];
              }
              closest_point(q, A, B, C, X);
              sub3(q, X, d);
              const double pen = R - sqrt(dot3(d, d));
              if (pen > best) { best = pen; bt = t; }
            }
            double tmin = INFINITY;
            int th = -1;
            const double D[3] = {-a[0], -a[1], -a[2]};
            for (int t = 0; t < nt; ++t) {   /* the ray's first crossing */
              double A[3], B[3], C[3], tt;
              for (int i = 0; i < 3; ++i) {
                A[i] = V[3 * TR[3 * t] + i]; B[i] = V[3 * TR[3 * t + 1] + i]; C[i] = V[3 * TR[3 * t + 2] + i];
              }
              if (ray_hit(q, D, A, B, C, &tt) && tt < tmin) { tmin = tt; th = t; }
            }
            if (th >= 0) {
              double A[3], B[3], C[3], n[3];
              for (int i = 0; i < 3; ++i) {
                A[i] = V[3 * TR[3 * th] + i]; B[i] = V[3 * TR[3 * th + 1] + i]; C[i] = V[3 * TR[3 * th + 2] + i];
              }
              face_normal(A, B, C, n);
              if (dot3(D, n) > 0.0 && R + tmin > best) { best = R + tmin; bt = th; }
            }
          }
          depth[(int64_t)s * ET + k] = best;
          tri[(int64_t)s * ET + k] = bt;
          double nl[3] = {0, 0, 0};
          if (bt >= 0) {
            double A[3], B[3], C[3], n[3], nw[3];
            for (int i = 0; i < 3; ++i) {
              A[i] = V[3 * TR[3 * bt] + i]; B[i] = V[3 * TR[3 * bt + 1] + i]; C[i] = V[3 * TR[3 * bt + 2] + i];
            }
            face_normal(A, B, C, n);
            for (int r = 0; r < 3; ++r) nw[r] = RO[r][0] * n[0] + RO[r][1] * n[1] + RO[r][2] * n[2];
            for (int r = 0; r < 3; ++r) nl[r] = RL[0][r] * nw[0] + RL[1][r] * nw[1] + RL[2][r] * nw[2];
          }
          for (int r = 0; r < 3; ++r) normal[((int64_t)s * 3 + r) * ET + k] = nl[r];
          if (tri_query && tri_pen_out) {
            const int tq = tri_query[(int64_t)s * ET + k];
            double pen = -INFINITY;
            if (tq >= 0 && tq < nt && R > 0) {
              double A[3], B[3], C[3];
              for (int i = 0; i < 3; ++i) {
                A[i] = V[3 * TR[3 * tq] + i]; B[i] = V[3 * TR[3 * tq + 1] + i]; C[i] = V[3 * TR[3 * tq + 2] + i];
              }
              pen = tri_pen(q, a, R, A, B, C);
            }
            tri_pen_out[(int64_t)s * ET + k] = pen;
          }
        }
      }
    }
}
