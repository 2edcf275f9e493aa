// ElastomerTaxel (App. A.7) behind include/tg_elastomer.h.
//
// Work layout.  One wave per (env, sensor link), persistent over the steps of a launch.  The
// object's tracked points are spread over the lanes (lane + 64 k, k < PPL) and their anchors
// stay in registers for the whole launch (read once, written once).  Per step:
//   1. poses (uniform loads), the object-change check;
//   2. the link's source probes with h_i > 0 go to an LDS list (ballot compaction);
//   3. the points: create sorts each cloud along a Morton curve and cuts it into chunks of 64
//      (chunk k = the k-th point of every lane) with a bounding sphere each.  Lane k places chunk
//      k's centre in the sensor frame; a chunk whose sphere stays farther than eta_exit from the
//      pad (pad SDF at the centre minus the radius, with a 1 um margin for rounding) can hold no
//      anchor and no contact, so its anchors are dropped, as the per-point rule would drop them,
//      and its points are skipped.  The other points get their sensor-frame position, pad SDF and
//      anchor update in the fixed FP32 sequence; points that are anchored and inside the pad go
//      to an LDS list, which is consumed into the markers' accumulators whenever it could
//      overflow (and at the end);
//   4. the markers: lane L serves marker L % nl with split L / nl of the terms (S = 64 / nl
//      splits), so a 20-marker fingertip keeps 60 lanes busy; the splits' partial sums meet in
//      LDS in split order, and the marker's lane writes y_j.
// All LDS regions belong to the one wave, so barriers are cheap.  The work is FP32 ALU (an
// exponential and about 30 operations per (marker, term)); the bytes are the points (L2),
// the depths of the link and the displacements out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/tg_elastomer.h"
#include "readout_device.h"

using namespace tg;

namespace {
thread_local std::string g_elast_create_error;
constexpr int EL_MAX_MARKERS = 64;
constexpr int EL_MAX_POINTS = 1024;
constexpr int EL_LIST = 128;        // contact-list capacity (two waves' worth of points)

struct ElastParams {
  int32_t E, L, T, Ls, n_obj, max_pts;
  float s_d, s_s, lambda_d, lambda_s, alpha, c, ginv, rinv, eps2, eta_enter, eta_exit;
  const int32_t* sensor_links;   // [Ls]
  const int32_t* link_off;       // [L+1]
  const float4* tax;             // [T] (x_j, R_j)
  const float4* nrm;             // [T] (n_j, 0)
  const float4* pad;             // [Ls][2] (centre, 0), (half, 0)
  const int32_t* cloud_off;      // [n_obj + 1]
  const float4* pts;             // object-frame points (x, y, z, 0), Morton order per object
  const int32_t* chunk_off;      // [n_obj + 1] first chunk of each object
  const float4* chunks;          // bounding sphere (centre, radius) of each run of 64 points
  float4* anchor;                // [E][Ls][max_pts] (e_p, active as 0 / 1)
  int32_t* last_oid;             // [E][Ls]
};

struct ElastLaunch {
  const float* link_state;  // [S][13][E*L]
  const float* obj_state;   // [S][13][E] or null
  const int32_t* obj_id;    // [S][E]
  const float* depth;       // [S][E][T]
  float* disp;              // [S][3][E][T]
  int32_t n_steps;
};

// the pad's exact box SDF, written out (no contraction) as the oracle writes it
__device__ __forceinline__ float pad_sdf(float z0, float z1, float z2, const float4& c, const float4& h) {
  const float q0 = fabsf(z0 - c.x) - h.x, q1 = fabsf(z1 - c.y) - h.y, q2 = fabsf(z2 - c.z) - h.z;
  const float m0 = fmaxf(q0, 0.0f), m1 = fmaxf(q1, 0.0f), m2 = fmaxf(q2, 0.0f);
  const float out = sqrtf(m0 * m0 + m1 * m1 + m2 * m2);
  const float in = fminf(fmaxf(q0, fmaxf(q1, q2)), 0.0f);
  return out + in;
}
__device__ __forceinline__ void tproj(float v0, float v1, float v2, float n0, float n1, float n2, float& o0,
                                      float& o1, float& o2) {
  const float d = fmaf(v2, n2, fmaf(v1, n1, v0 * n0));
  o0 = fmaf(-d, n0, v0);
  o1 = fmaf(-d, n1, v1);
  o2 = fmaf(-d, n2, v2);
}
}  // namespace

template <int PPL>
__global__ __launch_bounds__(64) void tg_elast_kernel(const ElastParams p, const ElastLaunch q) {
  __shared__ float4 src_a[EL_MAX_MARKERS], src_b[EL_MAX_MARKERS];   // (x_i, h_i), (h_i^alpha, ...)
  __shared__ float4 lst_a[EL_LIST], lst_b[EL_LIST];                 // (z_p, h_p), (z_p - e_p, 0)
  __shared__ float red[3][64];
  const int lane = threadIdx.x;
  const int e = blockIdx.x / p.Ls, li = blockIdx.x - e * p.Ls;
  const int l = p.sensor_links[li];
  const int j0 = p.link_off[l], nl = p.link_off[l + 1] - j0;
  const int64_t EL = (int64_t)p.E * p.L, ET = (int64_t)p.E * p.T;
  const float4 pc = p.pad[2 * li], ph = p.pad[2 * li + 1];
  // marker lanes: marker jj with split g of the terms
  const int S = nl > 0 ? 64 / nl : 1;
  const int jj = nl > 0 ? lane % nl : 0, g = nl > 0 ? lane / nl : 64;
  const bool mlane = g < S;
  float4 xj = make_float4(0.f, 0.f, 0.f, 0.f), nj = xj;
  if (mlane) {
    xj = p.tax[j0 + jj];
    nj = p.nrm[j0 + jj];
  }
  // anchors in registers
  const int64_t sl = (int64_t)e * p.Ls + li;
  float ax[PPL], ay[PPL], az[PPL];
  uint32_t act = 0;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int idx = lane + 64 * k;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    if (idx < p.max_pts) a = p.anchor[sl * p.max_pts + idx];
    ax[k] = a.x; ay[k] = a.y; az[k] = a.z;
    if (a.w != 0.f) act |= 1u << k;
  }
  int last = p.last_oid[sl];

  for (int s = 0; s < q.n_steps; ++s) {
    const int oid = q.obj_id[(int64_t)s * p.E + e];
    if (oid != last) {
      act = 0;
      last = oid;
    }
    const bool has = oid >= 0 && oid < p.n_obj;
    float RL[9], RO[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}, pO[3] = {0.f, 0.f, 0.f}, pL[3];
    {
      const float* ls = q.link_state + (int64_t)s * 13 * EL + (int64_t)e * p.L + l;
      pL[0] = ls[0]; pL[1] = ls[EL]; pL[2] = ls[2 * EL];
      quat_to_R(ls[3 * EL], ls[4 * EL], ls[5 * EL], ls[6 * EL], RL);
    }
    if (has && q.obj_state) {
      const float* os = q.obj_state + (int64_t)s * 13 * p.E + e;
      pO[0] = os[0]; pO[1] = os[p.E]; pO[2] = os[2 * p.E];
      quat_to_R(os[3 * p.E], os[4 * p.E], os[5 * p.E], os[6 * p.E], RO);
    }
    // 2. source probes with h_i > 0
    int nsrc = 0;
    {
      const float* dep = q.depth + (int64_t)s * ET + (int64_t)e * p.T + j0;
      float h = 0.f;
      float4 tx = make_float4(0.f, 0.f, 0.f, 0.f);
      if (lane < nl) {
        tx = p.tax[j0 + lane];
        h = fmaxf(dep[lane] - tx.w, 0.0f);
      }
      const bool on = lane < nl && h > 0.f;
      const uint64_t bal = __ballot(on);
      if (on) {
        const int slot = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        src_a[slot] = make_float4(tx.x, tx.y, tx.z, h);
        src_b[slot] = make_float4(powf(h, p.alpha), 0.f, 0.f, 0.f);
      }
      nsrc = __popcll(bal);
    }
    __syncthreads();
    // the marker accumulators, first with the dilation terms of this split
    float y0 = 0.f, y1 = 0.f, y2 = 0.f;
    if (mlane) {
      for (int i = g; i < nsrc; i += S) {
        const float4 a = src_a[i];
        float r0, r1, r2;
        tproj(xj.x - a.x, xj.y - a.y, xj.z - a.z, nj.x, nj.y, nj.z, r0, r1, r2);
        const float rr = fmaf(r2, r2, fmaf(r1, r1, r0 * r0));
        const float gk = expf(-p.lambda_d * rr);
        float wk = p.c * gk * p.ginv;
        if (p.c != 1.f) wk = fmaf((1.f - p.c) * p.rinv, 1.0f / (rr + p.eps2), wk);
        wk = wk * a.w;
        const float ha = src_b[i].x * gk;
        y0 = fmaf(p.s_d, fmaf(r0, wk, nj.x * ha), y0);
        y1 = fmaf(p.s_d, fmaf(r1, wk, nj.y * ha), y1);
        y2 = fmaf(p.s_d, fmaf(r2, wk, nj.z * ha), y2);
      }
    }
    // 3. tracked points, their anchors, and the shear terms through the contact list
    const int np = has ? p.cloud_off[oid + 1] - p.cloud_off[oid] : 0;
    const float4* pts = p.pts + (has ? p.cloud_off[oid] : 0);
    uint32_t near = 0;
    {
      const int nch = (np + 63) >> 6;
      bool nr = false;
      if (lane < nch) {
        const float4 cs = p.chunks[p.chunk_off[oid] + lane];
        float w[3], d[3], zc[3];
        mat_vec(RO, cs.x, cs.y, cs.z, w);
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c] = (w[c] + pO[c]) - pL[c];
        mat_T_vec(RL, d[0], d[1], d[2], zc);
        nr = !(pad_sdf(zc[0], zc[1], zc[2], pc, ph) - cs.w > p.eta_exit + 1e-6f);
      }
      near = (uint32_t)__ballot(nr);
    }
    int cnt = 0;
    auto consume = [&]() {
      __syncthreads();
      if (mlane) {
        for (int i = g; i < cnt; i += S) {
          const float4 a = lst_a[i], b = lst_b[i];
          float t0, t1, t2, d0, d1, d2;
          tproj(b.x, b.y, b.z, nj.x, nj.y, nj.z, t0, t1, t2);
          tproj(xj.x - a.x, xj.y - a.y, xj.z - a.z, nj.x, nj.y, nj.z, d0, d1, d2);
          const float dd = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
          const float f = p.s_s * a.w * expf(-p.lambda_s * dd);
          y0 = fmaf(f, t0, y0);
          y1 = fmaf(f, t1, y1);
          y2 = fmaf(f, t2, y2);
        }
      }
      __syncthreads();
      cnt = 0;
    };
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      if (64 * k >= np) break;   // uniform: no points left for any lane
      if (!((near >> k) & 1u)) {  // uniform: the chunk is far from the pad
        act &= ~(1u << k);
        continue;
      }
      const int idx = lane + 64 * k;
      bool on = false;
      float z[3] = {0.f, 0.f, 0.f}, hp = 0.f;
      if (idx < np) {
        const float4 ph4 = pts[idx];
        float w[3], d[3];
        mat_vec(RO, ph4.x, ph4.y, ph4.z, w);
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c] = (w[c] + pO[c]) - pL[c];
        mat_T_vec(RL, d[0], d[1], d[2], z);
        const float phi = pad_sdf(z[0], z[1], z[2], pc, ph);
        const bool a = (act >> k) & 1u;
        if (!a && phi < -p.eta_enter) {
          act |= 1u << k;
          ax[k] = z[0]; ay[k] = z[1]; az[k] = z[2];
        } else if (a && phi > p.eta_exit) {
          act &= ~(1u << k);
        }
        hp = fmaxf(-phi, 0.0f);
        on = ((act >> k) & 1u) && hp > 0.f;
      }
      const uint64_t bal = __ballot(on);
      if (bal) {
        if (cnt + 64 > EL_LIST) consume();
        if (on) {
          const int slot = cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
          lst_a[slot] = make_float4(z[0], z[1], z[2], hp);
          lst_b[slot] = make_float4(z[0] - ax[k], z[1] - ay[k], z[2] - az[k], 0.f);
        }
        cnt += __popcll(bal);
      }
    }
    if (cnt > 0) consume();
    // 4. the splits meet in LDS, in split order
    if (mlane && g > 0) {
      red[0][lane] = y0; red[1][lane] = y1; red[2][lane] = y2;
    }
    __syncthreads();
    if (mlane && g == 0) {
      for (int gg = 1; gg < S; ++gg) {
        y0 += red[0][gg * nl + jj];
        y1 += red[1][gg * nl + jj];
        y2 += red[2][gg * nl + jj];
      }
      float* o = q.disp + (int64_t)s * 3 * ET + (int64_t)e * p.T + j0 + jj;
      o[0] = y0;
      o[ET] = y1;
      o[2 * ET] = y2;
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int idx = lane + 64 * k;
    if (idx < p.max_pts) p.anchor[sl * p.max_pts + idx] = make_float4(ax[k], ay[k], az[k], ((act >> k) & 1u) ? 1.f : 0.f);
  }
  if (lane == 0) p.last_oid[sl] = last;
}

__global__ void tg_elast_reset_kernel(float4* anchor, int32_t* last_oid, int64_t na, int64_t nl) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < na) anchor[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (i < nl) last_oid[i] = -2;
}

struct tg_elast {
  ElastParams p{};
  int ppl = 1;
  std::vector<void*> allocs;
  std::string err;
};

namespace {
tg_status efail(tg_elast* h, tg_status s, const std::string& msg) {
  if (h) h->err = msg; else g_elast_create_error = msg;
  return s;
}
template <class T>
hipError_t ealloc(tg_elast* h, T** ptr, size_t n) {
  void* q = nullptr;
  const hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
  if (e == hipSuccess) h->allocs.push_back(q);
  *ptr = (T*)q;
  return e;
}
bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }
hipError_t reset_state(const ElastParams& p, hipStream_t st) {
  const int64_t nl = (int64_t)p.E * p.Ls, na = nl * p.max_pts, n = std::max(na, nl);
  hipLaunchKernelGGL(tg_elast_reset_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p.anchor, p.last_oid,
                     na, nl);
  return hipGetLastError();
}
}  // namespace

extern "C" {

tg_status tg_elast_create(const tg_elast_config* cfg, tg_elast** out) {
  if (!out) return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!cfg) return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "cfg is NULL");
  if (cfg->abi_version != TG_ABI_VERSION) return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "abi_version mismatch");
  const int E = cfg->num_envs, L = cfg->num_links, T = cfg->num_taxels, NO = cfg->num_objects, Ls = cfg->num_sensor_links;
  if (E < 1 || L < 1 || T < 1 || NO < 0 || Ls < 1) return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "sizes must be positive");
  if (!cfg->link_taxel_offset || !cfg->taxel_pos || !cfg->taxel_normal || !cfg->taxel_radius || !cfg->sensor_links ||
      !cfg->pad_center || !cfg->pad_half || (NO > 0 && !cfg->clouds))
    return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "NULL array");
  if ((int64_t)E * T * 3 >= (int64_t(1) << 31)) return efail(nullptr, TG_ERR_UNSUPPORTED, "E * T * 3 exceeds 2^31");
  const int32_t* off = cfg->link_taxel_offset;
  if (off[0] != 0 || off[L] != T) return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "link offsets must run 0..T");
  for (int l = 0; l < L; ++l)
    if (off[l + 1] < off[l]) return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "link offsets decrease");
  const float prm[] = {cfg->s_d, cfg->s_s, cfg->lambda_d, cfg->lambda_s, cfg->alpha, cfg->c, cfg->eps, cfg->eta_enter,
                       cfg->eta_exit};
  for (float v : prm)
    if (!std::isfinite(v)) return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "non-finite parameter");
  if (!(cfg->lambda_d > 0.f) || !(cfg->lambda_s >= 0.f) || !(cfg->eps > 0.f) || !(cfg->c >= 0.f && cfg->c <= 1.f) ||
      !(cfg->alpha > 0.f) || !(cfg->eta_enter >= 0.f) || !(cfg->eta_exit >= 0.f))
    return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "parameter out of range");
  std::vector<int32_t> sls(Ls);
  std::vector<float4> pads(2 * Ls);
  for (int i = 0; i < Ls; ++i) {
    const int l = cfg->sensor_links[i];
    if (l < 0 || l >= L) return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "sensor link id out of range");
    const int n = off[l + 1] - off[l];
    if (n < 1) return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "sensor link without markers");
    if (n > EL_MAX_MARKERS) return efail(nullptr, TG_ERR_UNSUPPORTED, "sensor link of more than 64 markers");
    const float* c = cfg->pad_center + 3 * i;
    const float* hh = cfg->pad_half + 3 * i;
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(c[k]) || !(hh[k] > 0.f) || !std::isfinite(hh[k]))
        return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "pad box invalid");
    sls[i] = l;
    pads[2 * i] = make_float4(c[0], c[1], c[2], 0.f);
    pads[2 * i + 1] = make_float4(hh[0], hh[1], hh[2], 0.f);
  }
  std::vector<float4> tax(T), nrm(T);
  for (int j = 0; j < T; ++j) {
    tax[j] = make_float4(cfg->taxel_pos[3 * j], cfg->taxel_pos[3 * j + 1], cfg->taxel_pos[3 * j + 2], cfg->taxel_radius[j]);
    nrm[j] = make_float4(cfg->taxel_normal[3 * j], cfg->taxel_normal[3 * j + 1], cfg->taxel_normal[3 * j + 2], 0.f);
  }
  std::vector<int32_t> coff(NO + 1, 0), choff(NO + 1, 0);
  std::vector<float4> pts, chunks;
  int max_pts = 1;
  for (int o = 0; o < NO; ++o) {
    const tg_point_cloud& c = cfg->clouds[o];
    if (c.num_points < 0 || (c.num_points > 0 && !c.points))
      return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "cloud " + std::to_string(o) + " invalid");
    if (c.num_points > EL_MAX_POINTS) return efail(nullptr, TG_ERR_UNSUPPORTED, "cloud of more than 1024 points");
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int i = 0; i < c.num_points; ++i) {
      const float* x = c.points + 3 * (int64_t)i;
      if (!std::isfinite(x[0]) || !std::isfinite(x[1]) || !std::isfinite(x[2]))
        return efail(nullptr, TG_ERR_INVALID_ARGUMENT, "non-finite cloud point");
      for (int k = 0; k < 3; ++k) {
        lo[k] = i ? std::min(lo[k], (double)x[k]) : x[k];
        hi[k] = i ? std::max(hi[k], (double)x[k]) : x[k];
      }
    }
    // Morton order (10 bits per axis over the cloud's box), so each run of 64 points is compact
    std::vector<std::pair<uint32_t, int>> key(c.num_points);
    for (int i = 0; i < c.num_points; ++i) {
      uint32_t m = 0;
      for (int k = 0; k < 3; ++k) {
        const double u = hi[k] > lo[k] ? ((double)c.points[3 * (int64_t)i + k] - lo[k]) / (hi[k] - lo[k]) : 0.0;
        const uint32_t q = (uint32_t)std::min(1023.0, std::max(0.0, u * 1024.0));
        for (int b = 0; b < 10; ++b) m |= ((q >> b) & 1u) << (3 * b + k);
      }
      key[i] = {m, i};
    }
    std::sort(key.begin(), key.end());
    const size_t base = pts.size();
    for (int i = 0; i < c.num_points; ++i) {
      const float* x = c.points + 3 * (int64_t)key[i].second;
      pts.push_back(make_float4(x[0], x[1], x[2], 0.f));
    }
    // bounding sphere of each run of 64: centre = mean, radius = farthest point, rounded up
    for (int b0 = 0; b0 < c.num_points; b0 += 64) {
      const int b1 = std::min(c.num_points, b0 + 64);
      double m[3] = {0, 0, 0}, r = 0;
      for (int i = b0; i < b1; ++i) {
        m[0] += pts[base + i].x; m[1] += pts[base + i].y; m[2] += pts[base + i].z;
      }
      for (int k = 0; k < 3; ++k) m[k] /= (b1 - b0);
      const float mc[3] = {(float)m[0], (float)m[1], (float)m[2]};
      for (int i = b0; i < b1; ++i) {
        const double dx = pts[base + i].x - (double)mc[0], dy = pts[base + i].y - (double)mc[1],
                     dz = pts[base + i].z - (double)mc[2];
        r = std::max(r, std::sqrt(dx * dx + dy * dy + dz * dz));
      }
      chunks.push_back(make_float4(mc[0], mc[1], mc[2], (float)(r * (1.0 + 1e-6) + 1e-7)));
    }
    coff[o + 1] = coff[o] + c.num_points;
    choff[o + 1] = choff[o] + (c.num_points + 63) / 64;
    max_pts = std::max(max_pts, c.num_points);
  }
  const int ppl = max_pts <= 256 ? 4 : max_pts <= 512 ? 8 : 16;
  tg_elast* h = new (std::nothrow) tg_elast();
  if (!h) return efail(nullptr, TG_ERR_OUT_OF_MEMORY, "host allocation failed");
  ElastParams& p = h->p;
  p.E = E; p.L = L; p.T = T; p.Ls = Ls; p.n_obj = NO; p.max_pts = max_pts;
  p.s_d = cfg->s_d; p.s_s = cfg->s_s; p.lambda_d = cfg->lambda_d; p.lambda_s = cfg->lambda_s;
  p.alpha = cfg->alpha; p.c = cfg->c;
  p.ginv = (float)(std::sqrt(2.0 * (double)cfg->lambda_d) / std::exp(-0.5));   // 1 / g_bar
  p.rinv = (float)(2.0 * (double)cfg->eps);                                       // 1 / rho_bar
  p.eps2 = cfg->eps * cfg->eps;
  p.eta_enter = cfg->eta_enter; p.eta_exit = cfg->eta_exit;
  h->ppl = ppl;
  int32_t *dsl = nullptr, *doff = nullptr, *dcoff = nullptr, *dlast = nullptr, *dchoff = nullptr;
  float4 *dtax = nullptr, *dnrm = nullptr, *dpad = nullptr, *dpts = nullptr, *danc = nullptr, *dch = nullptr;
  const size_t nanc = (size_t)E * Ls * max_pts;
  hipError_t e = ealloc(h, &dsl, Ls);
  if (e == hipSuccess) e = ealloc(h, &doff, L + 1);
  if (e == hipSuccess) e = ealloc(h, &dtax, T);
  if (e == hipSuccess) e = ealloc(h, &dnrm, T);
  if (e == hipSuccess) e = ealloc(h, &dpad, 2 * Ls);
  if (e == hipSuccess) e = ealloc(h, &dcoff, NO + 1);
  if (e == hipSuccess) e = ealloc(h, &dpts, pts.size());
  if (e == hipSuccess) e = ealloc(h, &danc, nanc);
  if (e == hipSuccess) e = ealloc(h, &dlast, (size_t)E * Ls);
  if (e == hipSuccess) e = ealloc(h, &dchoff, NO + 1);
  if (e == hipSuccess) e = ealloc(h, &dch, chunks.size());
  if (e == hipSuccess) e = hipMemcpy(dchoff, choff.data(), (NO + 1) * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && !chunks.empty())
    e = hipMemcpy(dch, chunks.data(), chunks.size() * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dsl, sls.data(), Ls * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(doff, off, (L + 1) * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dtax, tax.data(), T * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dnrm, nrm.data(), T * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dpad, pads.data(), 2 * Ls * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dcoff, coff.data(), (NO + 1) * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && !pts.empty()) e = hipMemcpy(dpts, pts.data(), pts.size() * sizeof(float4), hipMemcpyHostToDevice);
  p.sensor_links = dsl; p.link_off = doff; p.tax = dtax; p.nrm = dnrm; p.pad = dpad; p.cloud_off = dcoff;
  p.pts = dpts; p.anchor = danc; p.last_oid = dlast; p.chunk_off = dchoff; p.chunks = dch;
  if (e == hipSuccess) e = reset_state(p, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    tg_elast_destroy(h);
    return efail(nullptr, TG_ERR_OUT_OF_MEMORY, std::string("device setup: ") + hipGetErrorString(e));
  }
  *out = h;
  return TG_OK;
}

tg_status tg_elast_rollout(tg_elast* h, const tg_step_inputs* in, const float* depth, float* disp, int32_t n_steps,
                           void* hip_stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->err.clear();
  if (!in || !depth || !disp) return efail(h, TG_ERR_INVALID_ARGUMENT, "inputs, depth or disp is NULL");
  if (n_steps < 0) return efail(h, TG_ERR_INVALID_ARGUMENT, "n_steps < 0");
  if (n_steps == 0) return TG_OK;
  if (!in->link_state || !in->obj_id) return efail(h, TG_ERR_INVALID_ARGUMENT, "link_state and obj_id are required");
  if (!aligned16(in->link_state) || !aligned16(in->obj_id) || (in->obj_state && !aligned16(in->obj_state)) ||
      !aligned16(depth) || !aligned16(disp))
    return efail(h, TG_ERR_INVALID_ARGUMENT, "pointers must be 16-byte aligned");
  ElastLaunch q{};
  q.link_state = in->link_state;
  q.obj_state = in->obj_state;
  q.obj_id = in->obj_id;
  q.depth = depth;
  q.disp = disp;
  q.n_steps = n_steps;
  const dim3 grid((unsigned)(h->p.E * h->p.Ls)), block(64);
  const hipStream_t st = (hipStream_t)hip_stream;
  switch (h->ppl) {
    case 4: hipLaunchKernelGGL(tg_elast_kernel<4>, grid, block, 0, st, h->p, q); break;
    case 8: hipLaunchKernelGGL(tg_elast_kernel<8>, grid, block, 0, st, h->p, q); break;
    default: hipLaunchKernelGGL(tg_elast_kernel<16>, grid, block, 0, st, h->p, q); break;
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? TG_OK : efail(h, TG_ERR_HIP, hipGetErrorString(e));
}

tg_status tg_elast_reset(tg_elast* h, void* hip_stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->err.clear();
  const hipError_t e = reset_state(h->p, (hipStream_t)hip_stream);
  return e == hipSuccess ? TG_OK : efail(h, TG_ERR_HIP, hipGetErrorString(e));
}

tg_status tg_elast_destroy(tg_elast* h) {
  if (!h) return TG_OK;
  for (void* ptr : h->allocs) (void)hipFree(ptr);
  delete h;
  return TG_OK;
}

const char* tg_elast_last_error(const tg_elast* h) { return h ? h->err.c_str() : g_elast_create_error.c_str(); }

}  // extern "C"
