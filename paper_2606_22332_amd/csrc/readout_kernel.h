// Device pieces of the tactile readout shared by the rollout, neural and thermal kernels: the
// parameter block (KParams) and launch arguments (KLaunch), the work-plan records (LinkInfo,
// LinkLds), and one probe's readout as a fixed FP32 sequence: probe transform -> trilinear
// lookup in the bricked grid SDF -> depth, contact bit, proximity -> for d > 0 the gradient
// normal, relative velocity and force/torque (App. A).
#pragma once
#include "readout_device.h"

namespace tg {

// One link of the hand as the kernel sees it.
struct LinkInfo {
  int32_t off, n;        // first taxel, taxel count
  int32_t envs;          // envs per block for this link
  int32_t nwin;          // 64-bit words spanned by [off, off+n)
  int32_t mt, kt, nt;    // dense crosstalk: M tiles of 16 rows, K tiles of 32, N tiles of 16 columns
  int32_t kp, kpd;       // padded K stride (bf16 elements) of the B staging, of the result staging
  int32_t afrag_off;     // first A tile of this link in the fragment buffer
  int32_t np;            // lanes per env: n rounded up to a multiple of 8 (aligned 8-lane groups)
};

// LDS carve-up (byte offsets), identical for every block of a launch.
struct LinkLds {
  int32_t pose, opose, oid, bits, sums, xz, tax, gtab, raw, bt, dt, afr, total;
};

struct KParams {
  // sizes
  int32_t E, L, T, n_obj, W;     // W = 64-bit words per env of a bit mask
  // constants
  const float4* taxA;            // [T] x_j (xyz), R_j
  const float4* taxB;            // [T] n_j (xyz), link index (int bits)
  const int32_t* link_off;       // [L+1]
  const GridDesc* grids;
  const float* grid_vals;
  float k_n, c_n, alpha, nk_t, k_w, mu, Rp, rpinv, eta_on, eta_off;
  int32_t alpha_is_one, spring_only;
  // noise
  uint32_t key0, key1;
  float drift_sigma, white_sigma, bias, quant, qinv;
  float kload, kunload, decay, beta;
  float two_rho, neg_rho;
  float chi;
  int32_t has_gain, has_stuck, has_radius;
  // noise state (library-owned)
  float* drift;                  // [6][E][T]
  float* hyst;                   // [6][E][T]
  float* hyst_prev;              // [6][E][T]
  uint8_t* schmitt;              // [E][T]
  uint8_t* dead;                 // [E][T]
  float* stuck;                  // [E][T]
  float* gain;                   // [E][T]
  // work items: one block per (link, env chunk)
  const int2* items;             // (link, first env)
  const LinkInfo* links;         // [L]
  int32_t n_items, n_items_pad;  // pad = multiple of 8 (XCD-aware remapping)
  int32_t gtab_lds;              // 1: grid descriptors staged in LDS
  int32_t afr_lds;               // 1: the link's dense crosstalk A fragments staged in LDS
  LinkLds lds;
  // dense crosstalk (kind 2)
  const uint4* xt_afrag;         // A fragments, 8 bf16 per lane, 64 lanes per 16x32 tile
  // device error word, read and cleared by the host: bit 0 = an object id outside
  // [-1, n_obj) was seen (that env was read out as having no object)
  uint32_t* err;
};

constexpr uint32_t DEVERR_BAD_OBJECT_ID = 1u;   // TG_DEVERR_BAD_OBJECT_ID of the C header

// Flag an object id outside [-1, n_obj) in the device error word.
__device__ __forceinline__ void check_object_id(uint32_t* err, int oid, int n_obj) {
  if (oid < -1 || oid >= n_obj) atomicOr(err, DEVERR_BAD_OBJECT_ID);
}

// Per-launch arguments (kernel arguments); everything fixed for a handle lives in a KParams
// copy in device memory that the kernel reads through an opaque pointer.
struct KLaunch {
  const KParams* kc;
  int32_t n_steps;
  int64_t step0;
  // inputs (per step strides implied by sizes)
  const float* link_state;       // [S][13][E*L]
  const float* obj_state;        // [S][13][E] or null
  const int32_t* obj_id;         // [S][E]
  // outputs (null = not requested)
  unsigned long long* bits;      // [S][E][W]
  unsigned long long* bits_noisy;
  float* depth;                  // [S][E][T]
  float* prox;
  float* surfdist;
  float* ft;                     // [S][6][E][T]
  float* ft_noisy;
  float* normal;                 // [S][3][E][T]
  float* link_sums;              // [S][11][L][E]
  float* link_sums_noisy;
};

struct TaxelOut {
  float depth, phi, prox, surf;
  float f[3], tau[3], mb[3];
  bool active, far;
};

// Probe centre in the world (q) and object (qo) frames (App. A.1, probe geometry).
__device__ __forceinline__ void probe_point(const Pose& Lp, const Pose* Op, const float xj[3], float q[3],
                                            float qo[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
    q[i] = fmaf(Lp.R[3 * i + 2], xj[2], fmaf(Lp.R[3 * i + 1], xj[1], fmaf(Lp.R[3 * i], xj[0], Lp.p[i])));
  if (Op) {
    mat_T_vec(Op->R, q[0] - Op->p[0], q[1] - Op->p[1], q[2] - Op->p[2], qo);
  } else {
    qo[0] = q[0]; qo[1] = q[1]; qo[2] = q[2];
  }
}

// Trilinear grid lookup: far flag, value (at the clamped point when far), the 8 corners and the
// cell coordinates for the lazily evaluated gradient, and the far-field surface distance.
struct GridHit {
  float phi, surf;
  float c000, c100, c010, c110, c001, c101, c011, c111;
  float t[3];
  bool far;
};
__device__ __forceinline__ void grid_lookup(const GridDesc& g, const float* grid_vals, const float qo[3], GridHit& h) {
  float u[3];
  bool far = false;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    u[i] = (qo[i] - g.origin[i]) * g.hinv;
    far |= !(u[i] >= 0.f && u[i] <= g.nm1);
  }
  float uc[3];
  int ii[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    uc[i] = far ? (u[i] > 0.f ? (u[i] < g.nm1 ? u[i] : g.nm1) : 0.f) : u[i];
    int k = (int)floorf(uc[i]);
    k = k > g.n - 2 ? g.n - 2 : k;
    ii[i] = k;
    h.t[i] = uc[i] - (float)k;
  }
  // Brick addressing, separable per axis (element units): x -> (x/4)*64 + x%4,
  // y -> (y/4)*64nb + (y%4)*4, z -> (z/4)*64nb^2 + (z%4)*16; the +1 corner steps into the next
  // brick when the cell sits on a brick's last row.  32-bit byte offsets from the uniform base of
  // all grids, so the loads use a scalar base.
  const uint32_t nb = (uint32_t)g.nb;
  const uint32_t x0 = (uint32_t)ii[0], y0 = (uint32_t)ii[1], z0 = (uint32_t)ii[2];
  const uint32_t sy = nb << 6, sz = sy * nb;
  const uint32_t ax0 = ((x0 >> 2) << 6) + (x0 & 3u);
  const uint32_t ax1 = ax0 + ((x0 & 3u) == 3u ? 61u : 1u);
  const uint32_t ay0 = (y0 >> 2) * sy + ((y0 & 3u) << 2);
  const uint32_t ay1 = ay0 + ((y0 & 3u) == 3u ? sy - 12u : 4u);
  const uint32_t az0 = (z0 >> 2) * sz + ((z0 & 3u) << 4);
  const uint32_t az1 = az0 + ((z0 & 3u) == 3u ? sz - 48u : 16u);
  const uint32_t base = (uint32_t)g.offset;
  const uint32_t r00 = base + ay0 + az0, r10 = base + ay1 + az0, r01 = base + ay0 + az1, r11 = base + ay1 + az1;
  const char* Gb = (const char*)grid_vals;
  h.c000 = *(const float*)(Gb + (r00 + ax0) * 4u); h.c100 = *(const float*)(Gb + (r00 + ax1) * 4u);
  h.c010 = *(const float*)(Gb + (r10 + ax0) * 4u); h.c110 = *(const float*)(Gb + (r10 + ax1) * 4u);
  h.c001 = *(const float*)(Gb + (r01 + ax0) * 4u); h.c101 = *(const float*)(Gb + (r01 + ax1) * 4u);
  h.c011 = *(const float*)(Gb + (r11 + ax0) * 4u); h.c111 = *(const float*)(Gb + (r11 + ax1) * 4u);
  const float* t = h.t;
  const float l00 = lerpf(t[0], h.c000, h.c100), l10 = lerpf(t[0], h.c010, h.c110);
  const float l01 = lerpf(t[0], h.c001, h.c101), l11 = lerpf(t[0], h.c011, h.c111);
  h.phi = lerpf(t[2], lerpf(t[1], l00, l10), lerpf(t[1], l01, l11));
  h.far = far;
  if (far) {
    const float du0 = u[0] - uc[0], du1 = u[1] - uc[1], du2 = u[2] - uc[2];
    h.surf = h.phi + sqrtf(fmaf(du2, du2, fmaf(du1, du1, du0 * du0))) * g.spacing;
  } else {
    h.surf = h.phi;
  }
}
// Gradient direction of the trilinear interpolant (the bilinear blend of the edge differences).
__device__ __forceinline__ void grid_grad(const GridHit& h, float& gx, float& gy, float& gz) {
  const float* t = h.t;
  gx = lerpf(t[2], lerpf(t[1], h.c100 - h.c000, h.c110 - h.c010), lerpf(t[1], h.c101 - h.c001, h.c111 - h.c011));
  gy = lerpf(t[2], lerpf(t[0], h.c010 - h.c000, h.c110 - h.c100), lerpf(t[0], h.c011 - h.c001, h.c111 - h.c101));
  gz = lerpf(t[1], lerpf(t[0], h.c001 - h.c000, h.c101 - h.c100), lerpf(t[0], h.c011 - h.c010, h.c111 - h.c110));
}

// Everything after the SDF: depth, proximity, and for d > 0 the contact normal (from the
// gradient direction `grad`, evaluated only then), relative velocity and force/torque
// (App. A, ContactDepthProbe, KinematicTaxel, ProximityTaxel).
template <class KP, class GradFn>
__device__ __forceinline__ void probe_finish(KP& p, const Pose& Lp, const Pose* Op, const float xj[3], float Rj,
                                             float4 tb, const float q[3], float phi, GradFn grad, TaxelOut& o) {
  o.phi = phi;
  const float diff = Rj - phi;
  const float d = diff > 0.f ? diff : 0.f;
  o.depth = d;
  {
    float w = (p.Rp - phi) * p.rpinv;
    w = w > 0.f ? (w < 1.f ? w : 1.f) : 0.f;
    o.prox = (w * w) * (3.0f - 2.0f * w);
  }
  if (!(d > 0.f)) return;
  float gx, gy, gz;
  grad(gx, gy, gz);
  const float n2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
  float m[3], mb[3];
  if (n2 > 0.f) {
    const float inv = 1.0f / sqrtf(n2);
    const float mh0 = gx * inv, mh1 = gy * inv, mh2 = gz * inv;
    if (Op) {
      mat_vec(Op->R, mh0, mh1, mh2, m);
    } else {
      m[0] = mh0; m[1] = mh1; m[2] = mh2;
    }
    mat_T_vec(Lp.R, m[0], m[1], m[2], mb);
  } else {
    float a[3];
    mat_vec(Lp.R, tb.x, tb.y, tb.z, a);
    m[0] = -a[0]; m[1] = -a[1]; m[2] = -a[2];
    mb[0] = -tb.x; mb[1] = -tb.y; mb[2] = -tb.z;
  }
  // relative point velocity in the link frame
  const float rL[3] = {q[0] - Lp.p[0], q[1] - Lp.p[1], q[2] - Lp.p[2]};
  float cw[3], dv[3], dw[3], vr[3];
  cross3(Lp.w, rL, cw);
  const float vLq[3] = {Lp.v[0] + cw[0], Lp.v[1] + cw[1], Lp.v[2] + cw[2]};
  if (Op) {
    const float rO[3] = {q[0] - Op->p[0], q[1] - Op->p[1], q[2] - Op->p[2]};
    float cwo[3];
    cross3(Op->w, rO, cwo);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      dv[i] = (Op->v[i] + cwo[i]) - vLq[i];
      dw[i] = Op->w[i] - Lp.w[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      dv[i] = -vLq[i];
      dw[i] = -Lp.w[i];
    }
  }
  mat_T_vec(Lp.R, dv[0], dv[1], dv[2], vr);
  const float s = p.alpha_is_one ? d : powf(d, p.alpha);
  float f[3], tau[3];
  if (p.spring_only) {
    const float Fn = p.k_n * s;
    f[0] = Fn * mb[0]; f[1] = Fn * mb[1]; f[2] = Fn * mb[2];
    cross3(xj, f, tau);
  } else {
    const float vn = fmaf(vr[2], mb[2], fmaf(vr[1], mb[1], vr[0] * mb[0]));
    float ft[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) ft[i] = p.nk_t * fmaf(-vn, mb[i], vr[i]);
    const float ks = p.k_n * s, cs = p.c_n * s;
    float Fn = fmaf(cs, vn, ks);
    Fn = Fn > 0.f ? Fn : 0.f;
    const float ftn2 = fmaf(ft[2], ft[2], fmaf(ft[1], ft[1], ft[0] * ft[0]));
    const float lim = p.mu * Fn;
    if (ftn2 > lim * lim) {
      const float sc = lim / sqrtf(ftn2);
      ft[0] = ft[0] * sc; ft[1] = ft[1] * sc; ft[2] = ft[2] * sc;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) f[i] = fmaf(Fn, mb[i], ft[i]);
    const float tw = fmaf(dw[2], m[2], fmaf(dw[1], m[1], dw[0] * m[0]));
    const float kt = p.k_w * tw;
    float cx[3];
    cross3(xj, f, cx);
#pragma unroll
    for (int i = 0; i < 3; ++i) tau[i] = fmaf(-kt, mb[i], cx[i]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) { o.f[i] = f[i]; o.tau[i] = tau[i]; o.mb[i] = mb[i]; }
}

__device__ __forceinline__ void taxel_out_clear(TaxelOut& o) {
  o.depth = 0.f; o.phi = 0.f; o.prox = 0.f; o.surf = 3.402823466e+38f;
#pragma unroll
  for (int i = 0; i < 3; ++i) { o.f[i] = 0.f; o.tau[i] = 0.f; o.mb[i] = 0.f; }
  o.active = false; o.far = false;
}

// Clean readout of one probe on the grid SDF; the operation sequence is fixed (see readout_device.h).
template <class KP>
__device__ __forceinline__ void readout_probe(KP& p, const GridDesc* gtab, const Pose& Lp, const Pose* Op, int oid,
                                              float4 ta, float4 tb, TaxelOut& o) {
  taxel_out_clear(o);
  const float Rj = ta.w;
  if (oid < 0 || oid >= p.n_obj || !(Rj > 0.f)) return;
  o.active = true;
  const float xj[3] = {ta.x, ta.y, ta.z};
  float q[3], qo[3];
  probe_point(Lp, Op, xj, q, qo);
  GridDesc g;
  if (p.gtab_lds) g = gtab[oid];
  else g = p.grids[oid];
  GridHit h;
  grid_lookup(g, p.grid_vals, qo, h);
  o.surf = h.surf;
  if (h.far) {
    o.far = true;
    return;
  }
  probe_finish(p, Lp, Op, xj, Rj, tb, q, h.phi, [&](float& gx, float& gy, float& gz) { grid_grad(h, gx, gy, gz); }, o);
}

}  // namespace tg
