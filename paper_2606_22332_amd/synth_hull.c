/* Exact signed distance to a convex polytope, used only to build synthetic
 * SDF grids (scene generation, not part of the readout).
 *
 * Inside, the distance to the boundary of a convex set is the largest plane
 * distance (all plane distances are <= 0 there).  Outside, the closest
 * boundary point lies on some face that faces the query point (positive plane
 * distance), so only those triangles are tested with the closest-point-on-
 * triangle routine of Ericson, "Real-Time Collision Detection", sec. 5.1.5.
 * Everything is FP64; the caller rounds the result once.
 */
#include <math.h>
#include <stdint.h>

static double dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void closest_on_triangle(const double* p, const double* a, const double* b, const double* c,
                                double* out) {
  double ab[3], ac[3], ap[3], bp[3], cp[3];
  for (int i = 0; i < 3; ++i) {
    ab[i] = b[i] - a[i];
    ac[i] = c[i] - a[i];
    ap[i] = p[i] - a[i];
    bp[i] = p[i] - b[i];
    cp[i] = p[i] - c[i];
  }
  double d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0 && d2 <= 0) { for (int i = 0; i < 3; ++i) out[i] = a[i]; return; }
  double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0 && d4 <= d3) { for (int i = 0; i < 3; ++i) out[i] = b[i]; return; }
  double vc = d1 * d4 - d3 * d2;
  if (vc <= 0 && d1 >= 0 && d3 <= 0) {
    double v = d1 / (d1 - d3);
    for (int i = 0; i < 3; ++i) out[i] = a[i] + v * ab[i];
    return;
  }
  double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0 && d5 <= d6) { for (int i = 0; i < 3; ++i) out[i] = c[i]; return; }
  double vb = d5 * d2 - d1 * d6;
  if (vb <= 0 && d2 >= 0 && d6 <= 0) {
    double w = d2 / (d2 - d6);
    for (int i = 0; i < 3; ++i) out[i] = a[i] + w * ac[i];
    return;
  }
  double va = d3 * d6 - d5 * d4;
  if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
    double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    for (int i = 0; i < 3; ++i) out[i] = b[i] + w * (c[i] - b[i]);
    return;
  }
  double den = 1.0 / (va + vb + vc);
  double v = vb * den, w = vc * den;
  for (int i = 0; i < 3; ++i) out[i] = a[i] + ab[i] * v + ac[i] * w;
}

/* points [n_pts][3]; verts [n_v][3]; tris [n_t][3] (indices); planes [n_t][4] = (unit normal, offset)
 * with n.x - offset = signed plane distance.  out [n_pts]. */
void hull_sdf_points(int64_t n_pts, const double* points, int n_v, const double* verts, int n_t,
                     const int32_t* tris, const double* planes, double* out) {
  (void)n_v;
  for (int64_t k = 0; k < n_pts; ++k) {
    const double* p = points + 3 * k;
    double smax = -INFINITY;
    for (int t = 0; t < n_t; ++t) {
      double s = dot(planes + 4 * t, p) - planes[4 * t + 3];
      if (s > smax) smax = s;
    }
    if (smax <= 0) { out[k] = smax; continue; }
    double best = INFINITY;
    for (int t = 0; t < n_t; ++t) {
      double s = dot(planes + 4 * t, p) - planes[4 * t + 3];
      if (s <= 0) continue;
      double q[3];
      closest_on_triangle(p, verts + 3 * tris[3 * t], verts + 3 * tris[3 * t + 1], verts + 3 * tris[3 * t + 2], q);
      double d[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
      double dd = dot(d, d);
      if (dd < best) best = dd;
    }
    out[k] = sqrt(best);
  }
}
