// Raycast contact-depth backend (App. A.1) behind include/tg_raycast.h.
//
// Data: per object a BVH over its triangles, built on the host by median splits along the
// longest axis of the triangle centroids (at most 4 triangles per leaf), boxes grown by a
// relative 1e-6 so FP32 rounding never culls a triangle the exact test would keep.  An interior
// node is one 64-byte record holding its two children's entries (box, and either the child's
// record or its leaf's first triangle and count), so one load gives both boxes and a child that
// fails its test is never loaded; each object's root entry is kept apart.  Triangles are stored
// in leaf order as (a, b, c, outward unit normal), 64 B each, with the mesh's own index.
//
// One thread per (step, env, probe), a block row per step.  The probe's centre and axis in the
// object frame, then two traversals, each descending into the nearer of
// two passing children and parking the other on a stack in LDS (one column per thread, so equal
// stack depths fall in different banks); leaves are tested as soon as their entry passes:
//   1. the sphere query: children within R - best of the centre, nearer box first; at a leaf the
//      closest point of each triangle (Voronoi regions of the triangle, with the hardware
//      reciprocal: 1 ulp); best penetration R - dist, the square root taken only for a triangle
//      closer than the bound;
//   2. the ray query along -a: children the ray enters before the nearest hit so far, nearer
//      entry first; at a leaf the ray-triangle test (Moller-Trumbore, barycentric slack 1e-6);
//      if the nearest hit leaves the mesh, R + t competes with the sphere's best.  It is skipped
//      for centres known to be outside (outside the object's box, or on the outer side of the
//      face holding the closest point), where its first crossing could only enter the mesh.
// Neighbouring lanes are neighbouring probes of one link, so their traversals visit nearly the
// same nodes (L2 hits; the meshes are a few hundred KB).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/tg_raycast.h"
#include "readout_device.h"

using namespace tg;

namespace {
thread_local std::string g_ray_create_error;
constexpr int RC_THREADS = 256;
constexpr int RC_STACK = 32;

struct RayNode {   // a child entry: an interior record's two children are entries 2 r and 2 r + 1
  float4 lo;   // box min; w: the child's record (interior) or its first triangle (leaf), as int bits
  float4 hi;   // box max; w: 0 (interior) or the leaf's triangle count, as int bits
};
struct RayTri {
  float4 a;    // w: the triangle's index in its mesh, as int bits
  float4 b;
  float4 c;
  float4 n;    // outward unit normal
};

struct RayParams {
  int32_t E, L, T, n_obj;
  const float4* tax_a;      // [T] (x_j, R_j)
  const float4* tax_b;      // [T] (n_j, link id as int bits)
  const RayNode* root;      // [n_obj] root entry of each object
  const RayNode* nodes;     // [2 * records] child entries
  const RayTri* tris;
};

struct RayLaunch {
  const float* link_state;  // [S][13][E*L]
  const float* obj_state;   // [S][13][E] or null
  const int32_t* obj_id;    // [S][E]
  float* depth;             // [S][E][T]
  float* normal;            // [S][3][E][T] or null
  int32_t* tri;             // [S][E][T] or null
  int32_t n_steps;
};

__device__ __forceinline__ float dot3f(float ax, float ay, float az, float bx, float by, float bz) {
  return fmaf(az, bz, fmaf(ay, by, ax * bx));
}
// squared distance from p to the closest point of triangle (a, b, c); face: whether that point
// lies inside the face (not on an edge or vertex).  The Voronoi region of the point (Ericson's
// tests, in his order of precedence) picks the closest point as a + v (b - a) + w (c - a) with
// v = nv / den and w = nw / den; the regions are selected without branches, so the lanes of a
// wave, whose probes fall in different regions, do not diverge, and one reciprocal serves them all.
__device__ float tri_dist2(float px, float py, float pz, const float4& a, const float4& b, const float4& c, bool& face) {
  const float abx = b.x - a.x, aby = b.y - a.y, abz = b.z - a.z;
  const float acx = c.x - a.x, acy = c.y - a.y, acz = c.z - a.z;
  const float apx = px - a.x, apy = py - a.y, apz = pz - a.z;
  const float d1 = dot3f(abx, aby, abz, apx, apy, apz), d2 = dot3f(acx, acy, acz, apx, apy, apz);
  const float bpx = px - b.x, bpy = py - b.y, bpz = pz - b.z;
  const float d3 = dot3f(abx, aby, abz, bpx, bpy, bpz), d4 = dot3f(acx, acy, acz, bpx, bpy, bpz);
  const float cpx = px - c.x, cpy = py - c.y, cpz = pz - c.z;
  const float d5 = dot3f(abx, aby, abz, cpx, cpy, cpz), d6 = dot3f(acx, acy, acz, cpx, cpy, cpz);
  const float vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
  const float e43 = d4 - d3, e56 = d5 - d6;
  // lowest precedence first: the face, then edge bc, edge ac, vertex c, edge ab, vertex b, vertex a
  float nv = vb, nw = vc, den = va + vb + vc;
  bool f = true;
  if (va <= 0.f && e43 >= 0.f && e56 >= 0.f) { nv = e56; nw = e43; den = e43 + e56; f = false; }   // edge bc
  if (vb <= 0.f && d2 >= 0.f && d6 <= 0.f) { nv = 0.f; nw = d2; den = d2 - d6; f = false; }        // edge ac
  if (d6 >= 0.f && d5 <= d6) { nv = 0.f; nw = 1.f; den = 1.f; f = false; }                        // vertex c
  if (vc <= 0.f && d1 >= 0.f && d3 <= 0.f) { nv = d1; nw = 0.f; den = d1 - d3; f = false; }        // edge ab
  if (d3 >= 0.f && d4 <= d3) { nv = 1.f; nw = 0.f; den = 1.f; f = false; }                        // vertex b
  if (d1 <= 0.f && d2 <= 0.f) { nv = 0.f; nw = 0.f; den = 1.f; f = false; }                       // vertex a
  face = f;
  const float inv = __builtin_amdgcn_rcpf(den), v = nv * inv, w = nw * inv;
  const float qx = fmaf(w, acx, fmaf(v, abx, a.x));
  const float qy = fmaf(w, acy, fmaf(v, aby, a.y));
  const float qz = fmaf(w, acz, fmaf(v, abz, a.z));
  const float dx = px - qx, dy = py - qy, dz = pz - qz;
  return dot3f(dx, dy, dz, dx, dy, dz);
}
// ray o + t d against triangle (a, b, c): t > 0 with barycentric slack 1e-6; returns t or +inf
__device__ float tri_ray(float ox, float oy, float oz, float dx, float dy, float dz, const float4& a, const float4& b,
                         const float4& c) {
  const float e1x = b.x - a.x, e1y = b.y - a.y, e1z = b.z - a.z;
  const float e2x = c.x - a.x, e2y = c.y - a.y, e2z = c.z - a.z;
  const float px = fmaf(dy, e2z, -(dz * e2y)), py = fmaf(dz, e2x, -(dx * e2z)), pz = fmaf(dx, e2y, -(dy * e2x));
  const float det = dot3f(e1x, e1y, e1z, px, py, pz);
  if (det == 0.f) return INFINITY;
  const float inv = __builtin_amdgcn_rcpf(det);
  const float tx = ox - a.x, ty = oy - a.y, tz = oz - a.z;
  const float u = dot3f(tx, ty, tz, px, py, pz) * inv;
  if (u < -1e-6f || u > 1.0f + 1e-6f) return INFINITY;
  const float qx = fmaf(ty, e1z, -(tz * e1y)), qy = fmaf(tz, e1x, -(tx * e1z)), qz = fmaf(tx, e1y, -(ty * e1x));
  const float v = dot3f(dx, dy, dz, qx, qy, qz) * inv;
  if (v < -1e-6f || u + v > 1.0f + 1e-6f) return INFINITY;
  const float t = dot3f(e2x, e2y, e2z, qx, qy, qz) * inv;
  return t > 0.f ? t : INFINITY;
}
}  // namespace

__global__ __launch_bounds__(RC_THREADS) void tg_ray_kernel(const RayParams p, const RayLaunch q) {
  __shared__ int32_t stk[RC_STACK * RC_THREADS];   // stk[depth * RC_THREADS + tid]
  const int tid = threadIdx.x;
  const int64_t ET = (int64_t)p.E * p.T, EL = (int64_t)p.E * p.L;
  const int64_t idx = (int64_t)blockIdx.x * RC_THREADS + tid;
  if (idx >= ET) return;   // (no barrier below: the stack column is the thread's own)
  const int e = (int)(idx / p.T), j = (int)(idx - (int64_t)e * p.T);
  const float4 ta = p.tax_a[j], tb = p.tax_b[j];
  const int l = __float_as_int(tb.w);
  const float R = ta.w;
  int32_t* st = stk + tid;
  // one step per block row (the steps are independent): many more waves than a loop over the
  // steps in each thread, so the chip fills and the divergent traversals balance out
  for (int s = blockIdx.y; s < q.n_steps; s += gridDim.y) {
    float v[7];
    const float* ls = q.link_state + (int64_t)s * 13 * EL + (int64_t)e * p.L + l;
#pragma unroll
    for (int c = 0; c < 7; ++c) v[c] = ls[c * EL];
    float RL[9];
    quat_to_R(v[3], v[4], v[5], v[6], RL);
    float x[3], a[3];
    mat_vec(RL, ta.x, ta.y, ta.z, x);
    mat_vec(RL, tb.x, tb.y, tb.z, a);
    const int oid = q.obj_id[(int64_t)s * p.E + e];
    const bool has = oid >= 0 && oid < p.n_obj;
    float RO[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}, pO[3] = {0.f, 0.f, 0.f};
    if (has && q.obj_state) {
      const float* os = q.obj_state + (int64_t)s * 13 * p.E + e;
      pO[0] = os[0]; pO[1] = os[p.E]; pO[2] = os[2 * p.E];
      quat_to_R(os[3 * p.E], os[4 * p.E], os[5 * p.E], os[6 * p.E], RO);
    }
    float best = 0.f;
    int bt = -1;
    if (has && R > 0.f) {
      float qo[3], ao[3];
      mat_T_vec(RO, (v[0] + x[0]) - pO[0], (v[1] + x[1]) - pO[1], (v[2] + x[2]) - pO[2], qo);
      mat_T_vec(RO, a[0], a[1], a[2], ao);
      const RayNode rt = p.root[oid];
      const float4 root_lo = rt.lo, root_hi = rt.hi;
      // 1. sphere query: children closer than R - best
      float lim = R;
      bool bface = false;
      auto sphere_tri = [&](int t) {
        const RayTri tr = p.tris[t];
        bool face;
        const float d2 = tri_dist2(qo[0], qo[1], qo[2], tr.a, tr.b, tr.c, face);
        if (d2 < lim * lim) {   // (the square root only for a deeper triangle)
          const float pen = R - sqrtf(d2);
          if (pen > best) {
            best = pen;
            bt = t;
            bface = face;
            lim = R - best;
          }
        }
      };
      auto sphere_leaf = [&](const RayNode& c) {
        const int w0 = __float_as_int(c.lo.w), cnt = __float_as_int(c.hi.w);
        for (int k = 0; k < cnt; ++k) sphere_tri(w0 + k);
      };
      auto box_d2 = [&](const RayNode& c) {
        const float ex = fmaxf(fmaxf(c.lo.x - qo[0], qo[0] - c.hi.x), 0.f);
        const float ey = fmaxf(fmaxf(c.lo.y - qo[1], qo[1] - c.hi.y), 0.f);
        const float ez = fmaxf(fmaxf(c.lo.z - qo[2], qo[2] - c.hi.z), 0.f);
        return dot3f(ex, ey, ez, ex, ey, ez);
      };
      int sp = 0;
      int cur = -1;
      if (box_d2(rt) < lim * lim) {
        if (__float_as_int(rt.hi.w) > 0) sphere_leaf(rt);
        else cur = __float_as_int(rt.lo.w);
      }
      while (cur >= 0) {
        const RayNode c0 = p.nodes[2 * cur], c1 = p.nodes[2 * cur + 1];
        const float d0 = box_d2(c0), d1 = box_d2(c1);
        const bool sw = d1 < d0;
        const RayNode& na = sw ? c1 : c0;
        const RayNode& nb = sw ? c0 : c1;
        const float da = sw ? d1 : d0, db = sw ? d0 : d1;
        int next = -1;
        if (da < lim * lim) {
          if (__float_as_int(na.hi.w) > 0) sphere_leaf(na);
          else next = __float_as_int(na.lo.w);
        }
        if (db < lim * lim) {   // (lim may have shrunk at the first child's leaf)
          if (__float_as_int(nb.hi.w) > 0) sphere_leaf(nb);
          else if (next < 0) next = __float_as_int(nb.lo.w);
          else st[sp++ * RC_THREADS] = __float_as_int(nb.lo.w);   // the host bounds the depth
        }
        if (next < 0 && sp > 0) next = st[--sp * RC_THREADS];
        cur = next;
      }
      // 2. ray query along -a: the nearest crossing.  It can only count when the centre is inside
      //    the mesh, so it is skipped when the centre is outside the object's box, or when its
      //    closest point lies inside a face and the centre is on that face's outer side (then the
      //    ray's first crossing enters the mesh).  Near the surface, where rounding could flip
      //    that side, the two tests agree to twice the centre's distance from the face.
      bool outside = !(qo[0] >= root_lo.x && qo[0] <= root_hi.x && qo[1] >= root_lo.y && qo[1] <= root_hi.y &&
                       qo[2] >= root_lo.z && qo[2] <= root_hi.z);
      if (!outside && bt >= 0 && bface) {
        const RayTri tr = p.tris[bt];
        outside = dot3f(qo[0] - tr.a.x, qo[1] - tr.a.y, qo[2] - tr.a.z, tr.n.x, tr.n.y, tr.n.z) > 0.f;
      }
      const float dx = -ao[0], dy = -ao[1], dz = -ao[2];
      const float ix = 1.0f / dx, iy = 1.0f / dy, iz = 1.0f / dz;
      float tmin = INFINITY;
      int th = -1;
      auto ray_tri = [&](int k) {
        const RayTri tr = p.tris[k];
        const float t = tri_ray(qo[0], qo[1], qo[2], dx, dy, dz, tr.a, tr.b, tr.c);
        if (t < tmin) {
          tmin = t;
          th = k;
        }
      };
      auto ray_leaf = [&](const RayNode& c) {
        const int w0 = __float_as_int(c.lo.w), cnt = __float_as_int(c.hi.w);
        for (int k = 0; k < cnt; ++k) ray_tri(w0 + k);
      };
      // entry parameter of the ray into a box, or +inf when it misses it before tmin
      auto box_t = [&](const RayNode& c) {
        const float t1x = (c.lo.x - qo[0]) * ix, t2x = (c.hi.x - qo[0]) * ix;
        const float t1y = (c.lo.y - qo[1]) * iy, t2y = (c.hi.y - qo[1]) * iy;
        const float t1z = (c.lo.z - qo[2]) * iz, t2z = (c.hi.z - qo[2]) * iz;
        const float tn = fmaxf(fmaxf(fminf(t1x, t2x), fminf(t1y, t2y)), fmaxf(fminf(t1z, t2z), 0.f));
        const float tf = fminf(fminf(fmaxf(t1x, t2x), fmaxf(t1y, t2y)), fminf(fmaxf(t1z, t2z), tmin));
        return tn <= tf ? tn : INFINITY;
      };
      sp = 0;
      cur = -1;
      if (!outside && box_t(rt) < INFINITY) {
        if (__float_as_int(rt.hi.w) > 0) ray_leaf(rt);
        else cur = __float_as_int(rt.lo.w);
      }
      while (cur >= 0) {
        const RayNode c0 = p.nodes[2 * cur], c1 = p.nodes[2 * cur + 1];
        const float t0 = box_t(c0), t1 = box_t(c1);
        const bool sw = t1 < t0;
        const RayNode& na = sw ? c1 : c0;
        const RayNode& nb = sw ? c0 : c1;
        const float ta_ = sw ? t1 : t0;
        int next = -1;
        if (ta_ < INFINITY) {
          if (__float_as_int(na.hi.w) > 0) ray_leaf(na);
          else next = __float_as_int(na.lo.w);
        }
        if (box_t(nb) < INFINITY) {   // (re-tested: tmin may have shrunk at the first child's leaf)
          if (__float_as_int(nb.hi.w) > 0) ray_leaf(nb);
          else if (next < 0) next = __float_as_int(nb.lo.w);
          else st[sp++ * RC_THREADS] = __float_as_int(nb.lo.w);
        }
        if (next < 0 && sp > 0) next = st[--sp * RC_THREADS];
        cur = next;
      }
      if (th >= 0) {
        const float4 n = p.tris[th].n;
        if (dot3f(dx, dy, dz, n.x, n.y, n.z) > 0.f && R + tmin > best) {
          best = R + tmin;
          bt = th;
        }
      }
    }
    const int64_t o = (int64_t)s * ET + idx;
    q.depth[o] = best;
    if (q.tri) q.tri[o] = bt >= 0 ? __float_as_int(p.tris[bt].a.w) : -1;
    if (q.normal) {
      float nl[3] = {0.f, 0.f, 0.f};
      if (bt >= 0) {
        const float4 n = p.tris[bt].n;
        float nw[3];
        mat_vec(RO, n.x, n.y, n.z, nw);
        mat_T_vec(RL, nw[0], nw[1], nw[2], nl);
      }
      float* nm = q.normal + (int64_t)s * 3 * ET + idx;
      nm[0] = nl[0];
      nm[ET] = nl[1];
      nm[2 * ET] = nl[2];
    }
  }
}

struct tg_ray {
  RayParams p{};
  std::vector<void*> allocs;
  std::string err;
};

namespace {
tg_status rfail(tg_ray* h, tg_status s, const std::string& msg) {
  if (h) h->err = msg; else g_ray_create_error = msg;
  return s;
}
template <class T>
hipError_t ralloc(tg_ray* h, T** ptr, size_t n) {
  void* q = nullptr;
  const hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
  if (e == hipSuccess) h->allocs.push_back(q);
  *ptr = (T*)q;
  return e;
}
bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }
float ibits(int v) {   // an int's bits as a float (the node and triangle tags)
  float f;
  std::memcpy(&f, &v, 4);
  return f;
}

// Median-split BVH over one mesh's triangles, appended to nodes / tris (depth first).
struct Builder {
  const float* V;
  const int32_t* F;
  std::vector<int> idx;
  std::vector<double> cen;   // [m][3]
  std::vector<RayNode>* nodes;
  std::vector<RayTri>* tris;
  int max_depth = 0;
  void box(int b, int e, double lo[3], double hi[3]) const {
    for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int i = b; i < e; ++i)
      for (int c = 0; c < 3; ++c)
        for (int k = 0; k < 3; ++k) {
          const double x = V[3 * F[3 * idx[i] + c] + k];
          lo[k] = std::min(lo[k], x);
          hi[k] = std::max(hi[k], x);
        }
  }
  // Returns the entry of the subtree over idx[b, e): its box and either its record (appended to
  // nodes as two child entries) or its leaf's triangles (appended to tris).
  RayNode build(int b, int e, int depth) {
    max_depth = std::max(max_depth, depth);
    RayNode me;
    double lo[3], hi[3];
    box(b, e, lo, hi);
    float flo[3], fhi[3];
    for (int k = 0; k < 3; ++k) {   // grown so FP32 rounding never culls a triangle
      const double g = 1e-6 * std::max(1.0, std::fabs(lo[k]) + std::fabs(hi[k])) + 1e-6 * (hi[k] - lo[k]);
      flo[k] = (float)(lo[k] - g);
      fhi[k] = (float)(hi[k] + g);
    }
    if (e - b <= 4) {
      const int first = (int)tris->size();
      for (int i = b; i < e; ++i) {
        const int t = idx[i];
        double P[3][3];
        for (int c = 0; c < 3; ++c)
          for (int k = 0; k < 3; ++k) P[c][k] = V[3 * F[3 * t + c] + k];
        double e1[3], e2[3], n[3];
        for (int k = 0; k < 3; ++k) { e1[k] = P[1][k] - P[0][k]; e2[k] = P[2][k] - P[0][k]; }
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double ln = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        RayTri tr;
        tr.a = make_float4((float)P[0][0], (float)P[0][1], (float)P[0][2], ibits(t));
        tr.b = make_float4((float)P[1][0], (float)P[1][1], (float)P[1][2], 0.f);
        tr.c = make_float4((float)P[2][0], (float)P[2][1], (float)P[2][2], 0.f);
        tr.n = make_float4((float)(n[0] / ln), (float)(n[1] / ln), (float)(n[2] / ln), 0.f);
        tris->push_back(tr);
      }
      me.lo = make_float4(flo[0], flo[1], flo[2], ibits(first));
      me.hi = make_float4(fhi[0], fhi[1], fhi[2], ibits(e - b));
      return me;
    }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = b; i < e; ++i)
      for (int k = 0; k < 3; ++k) {
        clo[k] = std::min(clo[k], cen[3 * idx[i] + k]);
        chi[k] = std::max(chi[k], cen[3 * idx[i] + k]);
      }
    int ax = 0;
    for (int k = 1; k < 3; ++k)
      if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
    const int mid = (b + e) / 2;
    std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e, [&](int u, int w) {
      return cen[3 * u + ax] < cen[3 * w + ax] || (cen[3 * u + ax] == cen[3 * w + ax] && u < w);
    });
    const int rec = (int)(nodes->size() / 2);
    nodes->push_back(RayNode{});
    nodes->push_back(RayNode{});
    const RayNode left = build(b, mid, depth + 1);
    const RayNode right = build(mid, e, depth + 1);
    (*nodes)[2 * (size_t)rec] = left;
    (*nodes)[2 * (size_t)rec + 1] = right;
    me.lo = make_float4(flo[0], flo[1], flo[2], ibits(rec));
    me.hi = make_float4(fhi[0], fhi[1], fhi[2], ibits(0));
    return me;
  }
};
}  // namespace

extern "C" {

tg_status tg_ray_create(const tg_ray_config* cfg, tg_ray** out) {
  if (!out) return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!cfg) return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "cfg is NULL");
  if (cfg->abi_version != TG_ABI_VERSION) return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "abi_version mismatch");
  const int E = cfg->num_envs, L = cfg->num_links, T = cfg->num_taxels, NO = cfg->num_objects;
  if (E < 1 || L < 1 || T < 1 || NO < 1) return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "sizes must be positive");
  if (!cfg->link_taxel_offset || !cfg->taxel_pos || !cfg->taxel_normal || !cfg->taxel_radius || !cfg->meshes)
    return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "NULL array");
  if ((int64_t)E * T * 3 >= (int64_t(1) << 31)) return rfail(nullptr, TG_ERR_UNSUPPORTED, "E * T * 3 exceeds 2^31");
  const int32_t* off = cfg->link_taxel_offset;
  if (off[0] != 0 || off[L] != T) return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "link offsets must run 0..T");
  std::vector<float4> ta(T), tb(T);
  for (int l = 0; l < L; ++l) {
    if (off[l + 1] < off[l]) return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "link offsets decrease");
    for (int j = off[l]; j < off[l + 1]; ++j) {
      const float r = cfg->taxel_radius[j];
      if (!(r >= 0.f) || !std::isfinite(r)) return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "invalid probe radius");
      ta[j] = make_float4(cfg->taxel_pos[3 * j], cfg->taxel_pos[3 * j + 1], cfg->taxel_pos[3 * j + 2], r);
      tb[j] = make_float4(cfg->taxel_normal[3 * j], cfg->taxel_normal[3 * j + 1], cfg->taxel_normal[3 * j + 2],
                          ibits(l));
    }
  }
  std::vector<RayNode> nodes;
  std::vector<RayTri> tris;
  std::vector<RayNode> roots(NO);
  for (int o = 0; o < NO; ++o) {
    const tg_mesh& m = cfg->meshes[o];
    if (m.num_verts < 3 || m.num_tris < 1 || !m.verts || !m.tris)
      return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "mesh " + std::to_string(o) + " invalid");
    if (m.num_tris > (1 << 20)) return rfail(nullptr, TG_ERR_UNSUPPORTED, "mesh of more than 2^20 triangles");
    for (int i = 0; i < 3 * m.num_verts; ++i)
      if (!std::isfinite(m.verts[i])) return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "non-finite vertex");
    Builder bd;
    bd.V = m.verts;
    bd.F = m.tris;
    bd.nodes = &nodes;
    bd.tris = &tris;
    bd.idx.resize(m.num_tris);
    std::iota(bd.idx.begin(), bd.idx.end(), 0);
    bd.cen.resize(3 * (size_t)m.num_tris);
    for (int t = 0; t < m.num_tris; ++t) {
      double P[3][3];
      for (int c = 0; c < 3; ++c) {
        const int vi = m.tris[3 * t + c];
        if (vi < 0 || vi >= m.num_verts) return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "vertex index out of range");
        for (int k = 0; k < 3; ++k) P[c][k] = m.verts[3 * vi + k];
      }
      double e1[3], e2[3];
      for (int k = 0; k < 3; ++k) { e1[k] = P[1][k] - P[0][k]; e2[k] = P[2][k] - P[0][k]; }
      const double nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2], nz = e1[0] * e2[1] - e1[1] * e2[0];
      if (!(nx * nx + ny * ny + nz * nz > 0.0)) return rfail(nullptr, TG_ERR_INVALID_ARGUMENT, "degenerate triangle");
      for (int k = 0; k < 3; ++k) bd.cen[3 * t + k] = (P[0][k] + P[1][k] + P[2][k]) / 3.0;
    }
    roots[o] = bd.build(0, m.num_tris, 0);
    if (bd.max_depth + 2 > RC_STACK) return rfail(nullptr, TG_ERR_UNSUPPORTED, "BVH deeper than the traversal stack");
  }
  tg_ray* h = new (std::nothrow) tg_ray();
  if (!h) return rfail(nullptr, TG_ERR_OUT_OF_MEMORY, "host allocation failed");
  RayParams& p = h->p;
  p.E = E; p.L = L; p.T = T; p.n_obj = NO;
  float4 *dta = nullptr, *dtb = nullptr;
  RayNode* droot = nullptr;
  RayNode* dn = nullptr;
  RayTri* dt = nullptr;
  hipError_t e = ralloc(h, &dta, T);
  if (e == hipSuccess) e = ralloc(h, &dtb, T);
  if (e == hipSuccess) e = ralloc(h, &droot, NO);
  if (e == hipSuccess) e = ralloc(h, &dn, nodes.size());
  if (e == hipSuccess) e = ralloc(h, &dt, tris.size());
  if (e == hipSuccess) e = hipMemcpy(dta, ta.data(), T * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dtb, tb.data(), T * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(droot, roots.data(), NO * sizeof(RayNode), hipMemcpyHostToDevice);
  if (e == hipSuccess && !nodes.empty())
    e = hipMemcpy(dn, nodes.data(), nodes.size() * sizeof(RayNode), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dt, tris.data(), tris.size() * sizeof(RayTri), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    tg_ray_destroy(h);
    return rfail(nullptr, TG_ERR_OUT_OF_MEMORY, std::string("device setup: ") + hipGetErrorString(e));
  }
  p.tax_a = dta; p.tax_b = dtb; p.root = droot; p.nodes = dn; p.tris = dt;
  *out = h;
  return TG_OK;
}

tg_status tg_ray_rollout(tg_ray* h, const tg_step_inputs* in, float* depth, float* normal, int32_t* tri,
                         int32_t n_steps, void* hip_stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->err.clear();
  if (!in || !depth) return rfail(h, TG_ERR_INVALID_ARGUMENT, "inputs or depth is NULL");
  if (n_steps < 0) return rfail(h, TG_ERR_INVALID_ARGUMENT, "n_steps < 0");
  if (n_steps == 0) return TG_OK;
  if (!in->link_state || !in->obj_id) return rfail(h, TG_ERR_INVALID_ARGUMENT, "link_state and obj_id are required");
  if (!aligned16(in->link_state) || !aligned16(in->obj_id) || (in->obj_state && !aligned16(in->obj_state)) ||
      !aligned16(depth) || (normal && !aligned16(normal)) || (tri && !aligned16(tri)))
    return rfail(h, TG_ERR_INVALID_ARGUMENT, "pointers must be 16-byte aligned");
  RayLaunch q{};
  q.link_state = in->link_state;
  q.obj_state = in->obj_state;
  q.obj_id = in->obj_id;
  q.depth = depth;
  q.normal = normal;
  q.tri = tri;
  q.n_steps = n_steps;
  const int64_t ET = (int64_t)h->p.E * h->p.T;
  hipLaunchKernelGGL(tg_ray_kernel, dim3((unsigned)((ET + RC_THREADS - 1) / RC_THREADS), (unsigned)std::min(n_steps, 65535)), dim3(RC_THREADS), 0,
                     (hipStream_t)hip_stream, h->p, q);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? TG_OK : rfail(h, TG_ERR_HIP, hipGetErrorString(e));
}

tg_status tg_ray_destroy(tg_ray* h) {
  if (!h) return TG_OK;
  for (void* ptr : h->allocs) (void)hipFree(ptr);
  delete h;
  return TG_OK;
}

const char* tg_ray_last_error(const tg_ray* h) { return h ? h->err.c_str() : g_ray_create_error.c_str(); }

}  // extern "C"
