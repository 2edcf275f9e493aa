// ProximityTaxel readout (App. A.6) behind include/tg_proximity.h.
//
// Per (env, taxel, step) the taxel sums, over the tracked object's surface points inside its
// sensing sphere, the penetration P_ij = R_j - |p_i - q_j| and its first moment P_ij (p_i - q_j).
// Every channel of the sensor follows from those two moments, because a point's velocity
// v_O + w_O x (p_i - p_O) is affine in its position:
//   sum P v_p  = S0 (v_O + w_O x (q_j - p_O)) + w_O x S1,      S0 = sum P,  S1 = sum P (p_i - q_j)
//   f   = k rho S0 a + k_s rho [V - a (V . a)],  V = sum P v_p - S0 v_tax
//   tau = k rho S1 x a
// The neighbour search runs in the object frame (distances are rotation invariant): each cloud is
// kept in a uniform cell grid, cell edge h = half the largest sensing radius, points sorted by
// cell, x fastest.  A probe visits the rows of cells (fixed y and z) that its sphere reaches; in
// each row the sphere's chord fixes the x-range of cells, one contiguous range of points.  Against
// cells as large as the radius (3 x 3 x 3 around the probe) this halves the points visited on the
// hand's workload (about 775 instead of 1450 per probe, 378 of them inside the sphere).  One thread
// per (step, env, taxel), a block row per step; neighbouring lanes hold neighbouring taxels of
// one link, so they walk nearly the same cells and their point loads hit the same L2 lines.  The
// visits are plain FP32 ALU work (a distance, a compare, the hardware square root and four
// multiply-adds per point inside the sphere).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/tg_proximity.h"
#include "readout_device.h"

using namespace tg;

namespace {
thread_local std::string g_prox_create_error;
constexpr int PX_THREADS = 256;

struct CloudDesc {      // one object's cell grid
  float origin[3];      // corner of cell (0,0,0), object frame
  float hinv;           // 1 / cell edge
  int32_t dims[3];      // cells per axis
  int32_t cell_off;     // first entry of this object's cell table (dims product + 1 entries)
  int32_t n_points;     // N_active of an env holding this object
  float h;              // cell edge
};

struct ProxParams {
  int32_t E, L, T, n_obj;
  float k, k_s, density, radius_rho, two_rho, neg_rho;
  uint32_t key0, key1;
  const float4* tax_a;      // [T] (x_j, R_j)
  const float4* tax_b;      // [T] (n_j, link id as float bits)
  const CloudDesc* clouds;  // [n_obj]
  const int32_t* cells;     // concatenated cell start tables (point index into pts)
  const float4* pts;        // sorted points (x, y, z, 0), object frame
};

struct ProxLaunch {
  const float* link_state;  // [S][13][E*L]
  const float* obj_state;   // [S][13][E] or null
  const int32_t* obj_id;    // [S][E]
  float* ft;                // [S][6][E][T]
  float* mass;              // [S][E][T] or null
  const float* gain;        // [E][T] or null
  int64_t step0;
  int32_t n_steps;
};
}  // namespace

__global__ __launch_bounds__(PX_THREADS) void tg_prox_kernel(const ProxParams p, const ProxLaunch q) {
  const int64_t ET = (int64_t)p.E * p.T, EL = (int64_t)p.E * p.L;
  const int64_t idx = (int64_t)blockIdx.x * PX_THREADS + threadIdx.x;
  if (idx >= ET) return;
  const int e = (int)(idx / p.T), j = (int)(idx - (int64_t)e * p.T);
  const float4 ta = p.tax_a[j], tb = p.tax_b[j];
  const int l = __float_as_int(tb.w);
  const float g = q.gain ? q.gain[idx] : 1.0f;
  // one step per block row (the steps are independent): the launch has n_steps times the waves of
  // a loop over the steps in each thread, so the chip fills and the divergent loops balance out
  for (int s = blockIdx.y; s < q.n_steps; s += gridDim.y) {
    float v[13];
    const float* ls = q.link_state + (int64_t)s * 13 * EL + (int64_t)e * p.L + l;
#pragma unroll
    for (int c = 0; c < 13; ++c) v[c] = ls[c * EL];
    float RL[9];
    quat_to_R(v[3], v[4], v[5], v[6], RL);
    float x[3], a[3], qv[3];
    mat_vec(RL, ta.x, ta.y, ta.z, x);            // R_L x_j (q_j - p_L)
    mat_vec(RL, tb.x, tb.y, tb.z, a);            // a_j
#pragma unroll
    for (int i = 0; i < 3; ++i) qv[i] = v[i] + x[i];
    const int oid = q.obj_id[(int64_t)s * p.E + e];
    float S0 = 0.f, S1[3] = {0.f, 0.f, 0.f};     // object frame moments
    float RO[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}, pO[3] = {0.f, 0.f, 0.f};
    float vO[3] = {0.f, 0.f, 0.f}, wO[3] = {0.f, 0.f, 0.f};
    int npts = 0;
    if (oid >= 0 && oid < p.n_obj) {
      if (q.obj_state) {
        float o[13];
        const float* os = q.obj_state + (int64_t)s * 13 * p.E + e;
#pragma unroll
        for (int c = 0; c < 13; ++c) o[c] = os[c * p.E];
        quat_to_R(o[3], o[4], o[5], o[6], RO);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          pO[i] = o[i];
          vO[i] = o[7 + i];
          wO[i] = o[10 + i];
        }
      }
      const CloudDesc cd = p.clouds[oid];
      npts = cd.n_points;
      float qo[3];
      mat_T_vec(RO, qv[0] - pO[0], qv[1] - pO[1], qv[2] - pO[2], qo);
      float R = ta.w;
      if (p.radius_rho > 0.f) {
        uint32_t x0 = (uint32_t)e, x1 = (uint32_t)j, x2 = (uint32_t)(q.step0 + s), x3 = 9u;
        philox4x32_10(x0, x1, x2, x3, p.key0, p.key1);
        R = R + fmaf(u01(x0), p.two_rho, p.neg_rho);
        R = R > 0.f ? R : 0.f;
      }
      const float R2 = R * R;
      // the culling below uses a radius grown by a relative 1e-5 (and 0.1 um), so rounding never
      // drops a row or cell that holds a point inside the sphere; the point test is exact
      const float Rc = fmaf(R, 1.00001f, 1e-7f), Rc2 = Rc * Rc;
      int lo[3], hi[3];
      bool empty = !(R > 0.f);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float u0 = (qo[i] - Rc - cd.origin[i]) * cd.hinv, u1 = (qo[i] + Rc - cd.origin[i]) * cd.hinv;
        // NaN or entirely outside the grid: no points in range
        if (!(u1 >= 0.f) || !(u0 < (float)cd.dims[i])) empty = true;
        lo[i] = u0 > 0.f ? (int)u0 : 0;
        hi[i] = u1 < (float)(cd.dims[i] - 1) ? (int)u1 : cd.dims[i] - 1;
      }
      if (!empty) {
        const int32_t* cs = p.cells + cd.cell_off;
        for (int cz = lo[2]; cz <= hi[2]; ++cz) {
          const float zl = fmaf((float)cz, cd.h, cd.origin[2]);
          const float ez = fmaxf(fmaxf(zl - qo[2], qo[2] - (zl + cd.h)), 0.f);
          for (int cy = lo[1]; cy <= hi[1]; ++cy) {
            const float yl = fmaf((float)cy, cd.h, cd.origin[1]);
            const float ey = fmaxf(fmaxf(yl - qo[1], qo[1] - (yl + cd.h)), 0.f);
            const float c2 = Rc2 - fmaf(ey, ey, ez * ez);
            if (!(c2 > 0.f)) continue;
            const float half = __builtin_amdgcn_sqrtf(c2);
            const float x0 = (qo[0] - half - cd.origin[0]) * cd.hinv, x1 = (qo[0] + half - cd.origin[0]) * cd.hinv;
            const int ax = x0 > (float)lo[0] ? (int)x0 : lo[0];
            const int bx = x1 < (float)hi[0] ? (int)x1 : hi[0];
            if (ax > bx) continue;
            const int row = (cz * cd.dims[1] + cy) * cd.dims[0];
            const int b = cs[row + ax], t = cs[row + bx + 1];
            for (int i = b; i < t; ++i) {
              const float4 pt = p.pts[i];
              const float dx = pt.x - qo[0], dy = pt.y - qo[1], dz = pt.z - qo[2];
              const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
              if (d2 < R2) {
                const float w = R - __builtin_amdgcn_sqrtf(d2);
                S0 += w;
                S1[0] = fmaf(w, dx, S1[0]);
                S1[1] = fmaf(w, dy, S1[1]);
                S1[2] = fmaf(w, dz, S1[2]);
              }
            }
          }
        }
      }
    }
    float f[3] = {0.f, 0.f, 0.f}, tau[3] = {0.f, 0.f, 0.f};
    if (npts > 0) {
      const float rho = p.density / (float)npts;
      float Sw[3];
      mat_vec(RO, S1[0], S1[1], S1[2], Sw);      // world-frame sum P (p_i - q_j)
      // relative velocity moment V = S0 (v_O + w_O x (q - p_O) - v_tax) + w_O x Sw
      float rq[3] = {qv[0] - pO[0], qv[1] - pO[1], qv[2] - pO[2]}, c1[3], c2[3], c3[3];
      cross3(wO, rq, c1);                        // w_O x (q - p_O)
      cross3(v + 10, x, c2);                     // w_L x (q - p_L)
      cross3(wO, Sw, c3);
      float V[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) V[i] = fmaf(S0, (vO[i] + c1[i]) - (v[7 + i] + c2[i]), c3[i]);
      const float vn = fmaf(V[2], a[2], fmaf(V[1], a[1], V[0] * a[0]));
      const float kr = p.k * rho, ksr = p.k_s * rho;
      float t3[3];
      cross3(Sw, a, t3);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        f[i] = fmaf(kr * S0, a[i], ksr * fmaf(-a[i], vn, V[i]));
        tau[i] = kr * t3[i];
      }
    }
    float fl[3], tl[3];
    mat_T_vec(RL, f[0], f[1], f[2], fl);
    mat_T_vec(RL, tau[0], tau[1], tau[2], tl);
    float* out = q.ft + (int64_t)s * 6 * ET + idx;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      __builtin_nontemporal_store(g * fl[i], out + i * ET);
      __builtin_nontemporal_store(g * tl[i], out + (3 + i) * ET);
    }
    if (q.mass) __builtin_nontemporal_store(S0, q.mass + (int64_t)s * ET + idx);
  }
}

struct tg_prox {
  ProxParams p{};
  std::vector<void*> allocs;
  std::string err;
};

namespace {
tg_status pfail(tg_prox* h, tg_status s, const std::string& msg) {
  if (h) h->err = msg; else g_prox_create_error = msg;
  return s;
}
template <class T>
hipError_t palloc(tg_prox* h, T** p, size_t n) {
  void* q = nullptr;
  const hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
  if (e == hipSuccess) h->allocs.push_back(q);
  *p = (T*)q;
  return e;
}
bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
}  // namespace

extern "C" {

tg_status tg_prox_create(const tg_prox_config* cfg, tg_prox** out) {
  if (!out) return pfail(nullptr, TG_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!cfg) return pfail(nullptr, TG_ERR_INVALID_ARGUMENT, "cfg is NULL");
  if (cfg->abi_version != TG_ABI_VERSION) return pfail(nullptr, TG_ERR_INVALID_ARGUMENT, "abi_version mismatch");
  const int E = cfg->num_envs, L = cfg->num_links, T = cfg->num_taxels, NO = cfg->num_objects;
  if (E < 1 || L < 1 || T < 1 || NO < 1) return pfail(nullptr, TG_ERR_INVALID_ARGUMENT, "sizes must be positive");
  if (!cfg->link_taxel_offset || !cfg->taxel_pos || !cfg->taxel_normal || !cfg->sensing_radius || !cfg->clouds)
    return pfail(nullptr, TG_ERR_INVALID_ARGUMENT, "NULL array");
  if ((int64_t)E * T * 6 >= (int64_t(1) << 31)) return pfail(nullptr, TG_ERR_UNSUPPORTED, "E * T * 6 exceeds 2^31");
  const int32_t* off = cfg->link_taxel_offset;
  if (off[0] != 0 || off[L] != T) return pfail(nullptr, TG_ERR_INVALID_ARGUMENT, "link offsets must run 0..T");
  for (int l = 0; l < L; ++l)
    if (off[l + 1] < off[l]) return pfail(nullptr, TG_ERR_INVALID_ARGUMENT, "link offsets decrease");
  if (!(cfg->radius_rho >= 0.f) || !(cfg->k >= 0.f) || !(cfg->k_s >= 0.f) || !(cfg->density >= 0.f))
    return pfail(nullptr, TG_ERR_INVALID_ARGUMENT, "negative constant");
  float rmax = 0.f;
  std::vector<float4> ta(T), tb(T);
  for (int l = 0; l < L; ++l)
    for (int j = off[l]; j < off[l + 1]; ++j) {
      const float r = cfg->sensing_radius[j];
      if (!(r >= 0.f)) return pfail(nullptr, TG_ERR_INVALID_ARGUMENT, "negative sensing radius");
      rmax = std::max(rmax, r);
      ta[j] = make_float4(cfg->taxel_pos[3 * j], cfg->taxel_pos[3 * j + 1], cfg->taxel_pos[3 * j + 2], r);
      int li = l;
      float lf;
      std::memcpy(&lf, &li, 4);
      tb[j] = make_float4(cfg->taxel_normal[3 * j], cfg->taxel_normal[3 * j + 1], cfg->taxel_normal[3 * j + 2], lf);
    }
  // cell edge: half the largest radius a query can take (radius noise included), at least 0.1 mm
  const float h = std::max(0.5f * (rmax + cfg->radius_rho), 1e-4f);
  std::vector<CloudDesc> cds(NO);
  std::vector<int32_t> cells;
  std::vector<float4> pts;
  for (int o = 0; o < NO; ++o) {
    const tg_point_cloud& c = cfg->clouds[o];
    if (c.num_points < 0 || (c.num_points > 0 && !c.points))
      return pfail(nullptr, TG_ERR_INVALID_ARGUMENT, "cloud " + std::to_string(o) + " invalid");
    CloudDesc& d = cds[o];
    float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
    for (int i = 0; i < c.num_points; ++i)
      for (int k = 0; k < 3; ++k) {
        const float x = c.points[3 * i + k];
        if (!std::isfinite(x)) return pfail(nullptr, TG_ERR_INVALID_ARGUMENT, "non-finite cloud point");
        lo[k] = i ? std::min(lo[k], x) : x;
        hi[k] = i ? std::max(hi[k], x) : x;
      }
    int64_t ncell = 1;
    for (int k = 0; k < 3; ++k) {
      d.origin[k] = lo[k];
      d.dims[k] = std::max(1, (int)std::floor((hi[k] - lo[k]) / h) + 1);
      ncell *= d.dims[k];
    }
    if (ncell > (int64_t(1) << 24)) return pfail(nullptr, TG_ERR_UNSUPPORTED, "cloud cell grid too large");
    d.hinv = 1.0f / h;
    d.cell_off = (int32_t)cells.size();
    d.n_points = c.num_points;
    d.h = h;
    // counting sort of the points by cell (x fastest)
    std::vector<int32_t> cid(c.num_points), cnt(ncell + 1, 0);
    for (int i = 0; i < c.num_points; ++i) {
      int ci[3];
      for (int k = 0; k < 3; ++k) {
        const int v = (int)((c.points[3 * i + k] - d.origin[k]) * d.hinv);
        ci[k] = std::min(std::max(v, 0), d.dims[k] - 1);
      }
      cid[i] = (ci[2] * d.dims[1] + ci[1]) * d.dims[0] + ci[0];
      ++cnt[cid[i] + 1];
    }
    for (int64_t k = 0; k < ncell; ++k) cnt[k + 1] += cnt[k];
    const int32_t base = (int32_t)pts.size();
    pts.resize(pts.size() + c.num_points);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int i = 0; i < c.num_points; ++i)
      pts[base + fill[cid[i]]++] = make_float4(c.points[3 * i], c.points[3 * i + 1], c.points[3 * i + 2], 0.f);
    for (int64_t k = 0; k <= ncell; ++k) cells.push_back(base + cnt[k]);
  }
  tg_prox* hd = new (std::nothrow) tg_prox();
  if (!hd) return pfail(nullptr, TG_ERR_OUT_OF_MEMORY, "host allocation failed");
  ProxParams& p = hd->p;
  p.E = E; p.L = L; p.T = T; p.n_obj = NO;
  p.k = cfg->k; p.k_s = cfg->k_s; p.density = cfg->density;
  p.radius_rho = cfg->radius_rho;
  p.two_rho = 2.0f * cfg->radius_rho;
  p.neg_rho = -cfg->radius_rho;
  p.key0 = (uint32_t)cfg->seed;
  p.key1 = (uint32_t)(cfg->seed >> 32);
  float4 *dta = nullptr, *dtb = nullptr, *dpts = nullptr;
  CloudDesc* dcd = nullptr;
  int32_t* dcells = nullptr;
  hipError_t e = palloc(hd, &dta, T);
  if (e == hipSuccess) e = palloc(hd, &dtb, T);
  if (e == hipSuccess) e = palloc(hd, &dcd, NO);
  if (e == hipSuccess) e = palloc(hd, &dcells, cells.size());
  if (e == hipSuccess) e = palloc(hd, &dpts, pts.size());
  if (e == hipSuccess) e = hipMemcpy(dta, ta.data(), T * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dtb, tb.data(), T * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dcd, cds.data(), NO * sizeof(CloudDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dcells, cells.data(), cells.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && !pts.empty()) e = hipMemcpy(dpts, pts.data(), pts.size() * sizeof(float4), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    tg_prox_destroy(hd);
    return pfail(nullptr, TG_ERR_OUT_OF_MEMORY, std::string("device setup: ") + hipGetErrorString(e));
  }
  p.tax_a = dta; p.tax_b = dtb; p.clouds = dcd; p.cells = dcells; p.pts = dpts;
  *out = hd;
  return TG_OK;
}

tg_status tg_prox_rollout(tg_prox* h, const tg_step_inputs* in, float* ft, float* mass, const float* gain,
                          int32_t n_steps, void* hip_stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->err.clear();
  if (!in || !ft) return pfail(h, TG_ERR_INVALID_ARGUMENT, "inputs or ft is NULL");
  if (n_steps < 0) return pfail(h, TG_ERR_INVALID_ARGUMENT, "n_steps < 0");
  if (n_steps == 0) return TG_OK;
  if (in->step < 0 || in->step + n_steps > (int64_t(1) << 32))
    return pfail(h, TG_ERR_INVALID_ARGUMENT, "steps must lie in [0, 2^32)");
  if (!in->link_state || !in->obj_id) return pfail(h, TG_ERR_INVALID_ARGUMENT, "link_state and obj_id are required");
  if (!aligned16(in->link_state) || !aligned16(in->obj_id) || (in->obj_state && !aligned16(in->obj_state)) ||
      !aligned16(ft) || (mass && !aligned16(mass)) || (gain && !aligned16(gain)))
    return pfail(h, TG_ERR_INVALID_ARGUMENT, "pointers must be 16-byte aligned");
  ProxLaunch q{};
  q.link_state = in->link_state;
  q.obj_state = in->obj_state;
  q.obj_id = in->obj_id;
  q.ft = ft;
  q.mass = mass;
  q.gain = gain;
  q.step0 = in->step;
  q.n_steps = n_steps;
  const int64_t ET = (int64_t)h->p.E * h->p.T;
  hipLaunchKernelGGL(tg_prox_kernel, dim3((unsigned)((ET + PX_THREADS - 1) / PX_THREADS), (unsigned)std::min(n_steps, 65535)),
                     dim3(PX_THREADS), 0,
                     (hipStream_t)hip_stream, h->p, q);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? TG_OK : pfail(h, TG_ERR_HIP, hipGetErrorString(e));
}

tg_status tg_prox_destroy(tg_prox* h) {
  if (!h) return TG_OK;
  for (void* p : h->allocs) (void)hipFree(p);
  delete h;
  return TG_OK;
}

const char* tg_prox_last_error(const tg_prox* h) { return h ? h->err.c_str() : g_prox_create_error.c_str(); }

}  // extern "C"
