// C-ABI implementation of the tactile readout library (include/tg_readout.h) and the
// kernel entry points.  Build: hipcc --offload-arch=gfx950 -O3 -ffp-contract=off
//   -fno-gpu-flush-denormals-to-zero -fhip-fp32-correctly-rounded-divide-sqrt -shared -fPIC
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/tg_readout.h"
#include "readout_kernel.h"
#include "xtalk_dense.h"

using namespace tg;

namespace {

thread_local std::string g_create_error;

constexpr int kSumCh = 10;   // value channels reduced per link

// LDS layout of the readout kernel (bytes), shared by host sizing and device carving.
struct LdsLayout {
  size_t pose, opose, oid, bits, sums, xt, xtb, xtx, total;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline LdsLayout lds_layout(int eb, int L, int T, int W, int noise, int xt, int tpad) {
  LdsLayout o;
  const size_t nr = (size_t)eb * T;
  size_t off = 0;
  o.pose = off; off = align16(off + 2 * (size_t)eb * L * sizeof(Pose));
  o.opose = off; off = align16(off + 2 * (size_t)eb * sizeof(Pose));
  o.oid = off; off = align16(off + 2 * (size_t)eb * sizeof(int));
  o.bits = off; off = align16(off + 2 * 2 * (size_t)eb * 2 * W * sizeof(unsigned));
  o.sums = off; off = align16(off + kSumCh * nr * sizeof(float));
  o.xt = off; off = align16(off + (xt == 1 ? 6 * nr * sizeof(float) : 0));
  o.xtb = off; off = align16(off + (xt == 2 ? 6 * (size_t)eb * tpad * sizeof(uint16_t) : 0));
  o.xtx = off; off = align16(off + (xt == 2 ? 6 * (size_t)eb * tpad * sizeof(float) : 0));
  o.total = off;
  (void)noise;
  return o;
}

}  // namespace

// ------------------------------------------------------------------------------------------------
// kernels
// ------------------------------------------------------------------------------------------------
template <int NOISE, int XT, int HY, int OBJ>
__global__ void __launch_bounds__(1024) tg_readout_kernel(const KParams p) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = p.T, L = p.L, eb = p.eb, W = p.W;
  const int nr = eb * T;
  const int e0 = blockIdx.x * eb;
  const int tid = threadIdx.x;
  const LdsLayout lay = lds_layout(eb, L, T, W, NOISE, XT, p.tpad);
  Pose* lpose = (Pose*)(smem + lay.pose);
  Pose* opose = (Pose*)(smem + lay.opose);
  int* oids = (int*)(smem + lay.oid);
  unsigned* bitw = (unsigned*)(smem + lay.bits);   // [parity][clean,noisy][eb][2W]
  float* sv = (float*)(smem + lay.sums);           // [10][nr]
  float* xv = (float*)(smem + lay.xt);             // [6][nr]

  const int el = tid / T;
  const int e = e0 + el;
  const bool act = tid < nr && e < p.E;
  const int j = act ? tid - el * T : 0;
  float4 ta = make_float4(0.f, 0.f, 0.f, 0.f), tb = ta;
  int lk = 0, la = 0, lb = 0;
  if (act) {
    ta = p.taxA[j];
    tb = p.taxB[j];
    lk = __float_as_int(tb.w);
    la = p.link_off[lk];
    lb = p.link_off[lk + 1];
  }
  const int64_t ET = (int64_t)p.E * T;
  const int64_t EL = (int64_t)p.E * L;
  const int64_t kk = (int64_t)e * T + j;
  const int words2 = 2 * W;

  // ---- noise state: registers for the whole launch
  float D[6] = {0, 0, 0, 0, 0, 0}, Y[6] = {0, 0, 0, 0, 0, 0}, XP[6] = {0, 0, 0, 0, 0, 0};
  bool sch = false, dead = false;
  float stuck = 0.f, gain = 1.f;
  if (NOISE && act) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if (p.drift_sigma != 0.f) D[c] = p.drift[c * ET + kk];
      if (HY) Y[c] = p.hyst[c * ET + kk];
      if (HY == 2) XP[c] = p.hyst_prev[c * ET + kk];
    }
    sch = p.schmitt[kk] != 0;
    dead = p.dead[kk] != 0;
    if (p.has_stuck) stuck = p.stuck[kk];
    if (p.has_gain) gain = p.gain[kk];
  }
  float gd[12], gw[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) { gd[i] = 0.f; gw[i] = 0.f; }
  if (XT == 2) {   // padding rows of the MFMA staging must read as zero
    uint32_t* xb = (uint32_t*)(smem + lay.xtb);
    for (int i = tid; i < 3 * eb * p.tpad; i += blockDim.x) xb[i] = 0u;
  }

  for (int s = 0; s < p.n_steps; ++s) {
    const int64_t t = p.step0 + s;
    const int par = s & 1;
    Pose* lp = lpose + par * eb * L;
    Pose* op = opose + par * eb;
    int* oi = oids + par * eb;
    unsigned* bw = bitw + par * 2 * eb * words2;
    unsigned* bwn = bw + eb * words2;
    // ---- stage link poses (one thread per (env, link)), object poses and ids
    {
      const float* ls = p.link_state + (int64_t)s * 13 * EL;
      for (int idx = tid; idx < eb * L; idx += blockDim.x) {
        if (e0 + idx / L < p.E) {
          const int64_t col = (int64_t)e0 * L + idx;
          float v[13];
#pragma unroll
          for (int c = 0; c < 13; ++c) v[c] = ls[c * EL + col];
          Pose P;
          quat_to_R(v[3], v[4], v[5], v[6], P.R);
#pragma unroll
          for (int i = 0; i < 3; ++i) { P.p[i] = v[i]; P.v[i] = v[7 + i]; P.w[i] = v[10 + i]; }
          lp[idx] = P;
        }
      }
      for (int idx = tid; idx < eb; idx += blockDim.x) {
        if (e0 + idx < p.E) {
          oi[idx] = p.obj_id[(int64_t)s * p.E + e0 + idx];
          if (OBJ) {
            const float* os = p.obj_state + (int64_t)s * 13 * p.E;
            float v[13];
#pragma unroll
            for (int c = 0; c < 13; ++c) v[c] = os[c * (int64_t)p.E + e0 + idx];
            Pose P;
            quat_to_R(v[3], v[4], v[5], v[6], P.R);
#pragma unroll
            for (int i = 0; i < 3; ++i) { P.p[i] = v[i]; P.v[i] = v[7 + i]; P.w[i] = v[10 + i]; }
            op[idx] = P;
          }
        }
      }
      for (int idx = tid; idx < 2 * eb * words2; idx += blockDim.x) bw[idx] = 0u;
    }
    __syncthreads();

    // ---- clean readout
    TaxelOut o;
    if (act) {
      readout_probe(p, lp[el * L + lk], OBJ ? &op[el] : nullptr, oi[el], ta, tb, o);
    } else {
      o.depth = 0.f; o.phi = 0.f; o.prox = 0.f; o.surf = 0.f; o.active = false; o.far = false;
#pragma unroll
      for (int i = 0; i < 3; ++i) { o.f[i] = 0.f; o.tau[i] = 0.f; o.mb[i] = 0.f; }
    }
    const bool bit = o.depth > p.eta_on;
    if (act) {
      const int64_t ok = (int64_t)s * ET + kk;
      if (p.depth) p.depth[ok] = o.depth;
      if (p.prox) p.prox[ok] = o.prox;
      if (p.surfdist) p.surfdist[ok] = o.surf;
      if (p.ft) {
        float* f = p.ft + (int64_t)s * 6 * ET + kk;
#pragma unroll
        for (int c = 0; c < 3; ++c) { f[c * ET] = o.f[c]; f[(c + 3) * ET] = o.tau[c]; }
      }
      if (p.normal) {
        float* nm = p.normal + (int64_t)s * 3 * ET + kk;
#pragma unroll
        for (int c = 0; c < 3; ++c) nm[c * ET] = o.mb[c];
      }
      if (bit) atomicOr(&bw[el * words2 + (j >> 5)], 1u << (j & 31));
    }
    const bool sums = p.link_sums != nullptr;
    if (sums && tid < nr) {
      sv[0 * nr + tid] = o.f[0]; sv[1 * nr + tid] = o.f[1]; sv[2 * nr + tid] = o.f[2];
      sv[3 * nr + tid] = o.tau[0]; sv[4 * nr + tid] = o.tau[1]; sv[5 * nr + tid] = o.tau[2];
      sv[6 * nr + tid] = bit ? 1.f : 0.f;
      sv[7 * nr + tid] = o.depth * tb.z;
      sv[8 * nr + tid] = o.depth * tb.y;
      sv[9 * nr + tid] = o.depth * tb.x;
    }
    float z[6] = {gain * o.f[0], gain * o.f[1], gain * o.f[2], gain * o.tau[0], gain * o.tau[1], gain * o.tau[2]};
    if (NOISE && XT == 1) {
      if (tid < nr) {
#pragma unroll
        for (int c = 0; c < 6; ++c) xv[c * nr + tid] = z[c];
      }
    }
    __syncthreads();
    if (p.bits) {
      for (int idx = tid; idx < eb * W; idx += blockDim.x) {
        const int e_ = e0 + idx / W;
        if (e_ < p.E)
          p.bits[(int64_t)s * p.E * W + (int64_t)e0 * W + idx] =
              (unsigned long long)bw[2 * idx] | ((unsigned long long)bw[2 * idx + 1] << 32);
      }
    }
    if (sums) link_sums_from_lds(p, sv, nr, e0, p.link_sums + (int64_t)s * 11 * EL);

    if (NOISE) {
      // ---- spatial crosstalk within the link
      float zt[6];
      if (XT == 1) {
        const float chi = p.chi;
        const bool hasl = j > la, hasr = j < lb - 1;
        const float cjj = 1.0f - chi * (float)((int)hasl + (int)hasr);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          float acc = cjj * z[c];
          if (act && hasl) acc = fmaf(chi, xv[c * nr + tid - 1], acc);
          if (act && hasr) acc = fmaf(chi, xv[c * nr + tid + 1], acc);
          zt[c] = acc;
        }
      } else if (XT == 2) {
        xtalk_dense_block(p, z, zt, smem + lay.xtb, smem + lay.xtx, el, j, lk, act, e0);
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) zt[c] = z[c];
      }
      // ---- random streams for this step
      if (p.drift_sigma != 0.f && ((t & 1) == 0 || s == 0) && act)
        gauss12(p.key0, p.key1, (uint32_t)e, (uint32_t)j, (uint32_t)(t >> 1), 0u, gd);
      if (p.white_sigma != 0.f && ((t & 1) == 0 || s == 0) && act)
        gauss12(p.key0, p.key1, (uint32_t)e, (uint32_t)j, (uint32_t)(t >> 1), 3u, gw);
      const bool hi = (t & 1) != 0;
      float fo[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const float x = zt[c];
        float h = x;
        if (HY == 1) {
          const float kap = fabsf(x) > fabsf(Y[c]) ? p.kload : p.kunload;
          Y[c] = fmaf(kap, x - Y[c], Y[c]);
          h = Y[c];
        } else if (HY == 2) {
          Y[c] = fmaf(p.decay, Y[c], x - XP[c]);
          XP[c] = x;
          h = fmaf(p.beta, Y[c], x);
        }
        float v = h;
        if (p.bias != 0.f) v = v + p.bias;
        if (p.white_sigma != 0.f) v = fmaf(p.white_sigma, hi ? gw[6 + c] : gw[c], v);
        if (p.drift_sigma != 0.f) {
          D[c] = fmaf(p.drift_sigma, hi ? gd[6 + c] : gd[c], D[c]);
          v = v + D[c];
        }
        if (p.quant > 0.f) v = p.quant * rintf(v * p.qinv);
        if (dead) v = stuck;
        fo[c] = v;
      }
      if (act && p.ft_noisy) {
        float* f = p.ft_noisy + (int64_t)s * 6 * ET + kk;
#pragma unroll
        for (int c = 0; c < 6; ++c) f[c * ET] = fo[c];
      }
      // ---- noisy contact bit: probe-radius noise, Schmitt hysteresis, dead overwrite
      float dd = o.depth;
      if (p.has_radius) {
        dd = 0.f;
        if (act && o.active && !o.far) {
          uint32_t x0 = (uint32_t)e, x1 = (uint32_t)j, x2 = (uint32_t)t, x3 = 6u;
          philox4x32_10(x0, x1, x2, x3, p.key0, p.key1);
          const float u = u01(x0);
          float Rn = ta.w + fmaf(u, p.two_rho, p.neg_rho);
          Rn = Rn > 0.f ? Rn : 0.f;
          const float df = Rn - o.phi;
          dd = df > 0.f ? df : 0.f;
        }
      }
      bool nb = (dd > p.eta_on) || (sch && dd > p.eta_off);
      if (dead) { nb = false; dd = 0.f; }
      sch = nb;
      if (act && nb) atomicOr(&bwn[el * words2 + (j >> 5)], 1u << (j & 31));
      const bool sums_n = p.link_sums_noisy != nullptr;
      if (sums_n) {
        __syncthreads();   // clean reduction has finished reading sv
      }
      if (sums_n && tid < nr) {
        sv[0 * nr + tid] = fo[0]; sv[1 * nr + tid] = fo[1]; sv[2 * nr + tid] = fo[2];
        sv[3 * nr + tid] = fo[3]; sv[4 * nr + tid] = fo[4]; sv[5 * nr + tid] = fo[5];
        sv[6 * nr + tid] = nb ? 1.f : 0.f;
        sv[7 * nr + tid] = dd * tb.z;
        sv[8 * nr + tid] = dd * tb.y;
        sv[9 * nr + tid] = dd * tb.x;
      }
      __syncthreads();
      if (p.bits_noisy) {
        for (int idx = tid; idx < eb * W; idx += blockDim.x) {
          const int e_ = e0 + idx / W;
          if (e_ < p.E)
            p.bits_noisy[(int64_t)s * p.E * W + (int64_t)e0 * W + idx] =
                (unsigned long long)bwn[2 * idx] | ((unsigned long long)bwn[2 * idx + 1] << 32);
        }
      }
      if (sums_n) link_sums_from_lds(p, sv, nr, e0, p.link_sums_noisy + (int64_t)s * 11 * EL);
    }
  }
  // ---- write the noise state back
  if (NOISE && act) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if (p.drift_sigma != 0.f) p.drift[c * ET + kk] = D[c];
      if (HY) p.hyst[c * ET + kk] = Y[c];
      if (HY == 2) p.hyst_prev[c * ET + kk] = XP[c];
    }
    p.schmitt[kk] = sch ? 1 : 0;
  }
}

// Episode reset: zero the dynamic state and draw dead flag, stuck value and gain with
// counter (env, taxel, reset step, 7).
__global__ void tg_reset_kernel(KParams p, const uint8_t* mask, int64_t step, float stuck_lo, float stuck_span,
                                float gain_lo, float gain_span, unsigned long long dead_thr) {
  const int64_t ET = (int64_t)p.E * p.T;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ET) return;
  const int e = (int)(k / p.T), j = (int)(k - (int64_t)e * p.T);
  if (mask && !mask[e]) return;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    p.drift[c * ET + k] = 0.f;
    p.hyst[c * ET + k] = 0.f;
    p.hyst_prev[c * ET + k] = 0.f;
  }
  p.schmitt[k] = 0;
  uint32_t x0 = (uint32_t)e, x1 = (uint32_t)j, x2 = (uint32_t)step, x3 = 7u;
  philox4x32_10(x0, x1, x2, x3, p.key0, p.key1);
  p.dead[k] = (unsigned long long)x0 < dead_thr ? 1 : 0;
  p.stuck[k] = fmaf(u01(x1), stuck_span, stuck_lo);
  p.gain[k] = fmaf(u01(x2), gain_span, gain_lo);
}

// ------------------------------------------------------------------------------------------------
// handle
// ------------------------------------------------------------------------------------------------
struct tg_readout {
  tg_readout_config cfg{};
  int E = 0, L = 0, T = 0, n_obj = 0, W = 0;
  int eb = 1, threads = 64;
  size_t lds = 0;
  int xt = 0, hy = 0, noise = 0;
  KParams kp{};
  std::vector<void*> allocs;
  std::string err;
  float stuck_lo = 0, stuck_span = 0, gain_lo = 1, gain_span = 0;
  unsigned long long dead_thr = 0;
  size_t state_bytes = 0;
  XtDense xtd;
};

namespace {

tg_status fail(tg_readout* h, tg_status s, const std::string& msg) {
  if (h) h->err = msg; else g_create_error = msg;
  return s;
}

template <class T>
hipError_t dalloc(tg_readout* h, T** p, size_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) h->allocs.push_back(q);
  *p = (T*)q;
  return e;
}

using KernelFn = void (*)(const KParams);

template <int N, int X, int Y, int O>
KernelFn pick() { return tg_readout_kernel<N, X, Y, O>; }

KernelFn select_kernel(int noise, int xt, int hy, int obj) {
  if (!noise) return obj ? pick<0, 0, 0, 1>() : pick<0, 0, 0, 0>();
#define TG_PICK(X, Y)                                                   \
  if (xt == X && hy == Y) return obj ? pick<1, X, Y, 1>() : pick<1, X, Y, 0>();
  TG_PICK(0, 0) TG_PICK(0, 1) TG_PICK(0, 2)
  TG_PICK(1, 0) TG_PICK(1, 1) TG_PICK(1, 2)
  TG_PICK(2, 0) TG_PICK(2, 1) TG_PICK(2, 2)
#undef TG_PICK
  return nullptr;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

extern "C" {

const char* tg_status_string(tg_status s) {
  switch (s) {
    case TG_OK: return "ok";
    case TG_ERR_INVALID_ARGUMENT: return "invalid argument";
    case TG_ERR_OUT_OF_MEMORY: return "out of device memory";
    case TG_ERR_HIP: return "HIP runtime error";
    case TG_ERR_UNSUPPORTED: return "unsupported configuration";
    case TG_ERR_UNSTABLE: return "unstable configuration";
    case TG_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* tg_readout_last_error(const tg_readout* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

tg_status tg_readout_destroy(tg_readout* h) {
  if (!h) return TG_OK;
  (void)hipDeviceSynchronize();
  for (void* p : h->allocs) (void)hipFree(p);
  for (void* p : h->xtd.allocs) (void)hipFree(p);
  delete h;
  return TG_OK;
}

tg_status tg_readout_create(const tg_readout_config* cfg, tg_readout** out) {
  g_create_error.clear();
  if (!out) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "cfg is NULL");
  if (cfg->abi_version != TG_ABI_VERSION) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "abi_version mismatch");
  const int E = cfg->num_envs, L = cfg->num_links, T = cfg->num_taxels, NO = cfg->num_objects;
  if (E <= 0 || L <= 0 || T <= 0 || NO <= 0) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "sizes must be positive");
  if (T > 1024) return fail(nullptr, TG_ERR_UNSUPPORTED, "more than 1024 taxels per env");
  if (!cfg->link_taxel_offset || !cfg->taxel_pos || !cfg->taxel_normal || !cfg->taxel_radius || !cfg->grids)
    return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "NULL host array in config");
  const int32_t* off = cfg->link_taxel_offset;
  if (off[0] != 0 || off[L] != T) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "link offsets must span [0, T]");
  for (int l = 0; l < L; ++l)
    if (off[l + 1] < off[l]) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "link offsets not monotone");
  for (int g = 0; g < NO; ++g) {
    const tg_sdf_grid& G = cfg->grids[g];
    if (G.n < 2 || !(G.spacing > 0.f) || !G.values) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "bad grid");
  }
  for (int j = 0; j < T; ++j)
    if (!(cfg->taxel_radius[j] >= 0.f)) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "negative taxel radius");
  if (!(cfg->prox_range > 0.f) || !(cfg->eta_on >= 0.f) || !(cfg->mu >= 0.f))
    return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "bad force/proximity parameters");
  const tg_noise_desc& nz = cfg->noise;
  const int noise = cfg->noise_enabled ? 1 : 0;
  if (noise) {
    if (!(nz.eta_off <= cfg->eta_on) || !(nz.eta_off >= 0.f))
      return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "need 0 <= eta_off <= eta_on");
    if (nz.hyst_mode < 0 || nz.hyst_mode > 2) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "hyst_mode");
    if (nz.hyst_mode == 1 && !(nz.tau_load_steps > 0.f && nz.tau_unload_steps > 0.f))
      return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "lag time constants must be positive");
    if (nz.hyst_mode == 2 && !(nz.maxwell_tau_s > 0.f && nz.dt_s > 0.f))
      return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "Maxwell tau and dt must be positive");
    if (nz.xtalk_kind < 0 || nz.xtalk_kind > 2) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "xtalk_kind");
    if (!(nz.p_dead >= 0.f && nz.p_dead <= 1.f)) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "p_dead");
    if (!(nz.stuck_lo <= nz.stuck_hi) || !(nz.gain_lo <= nz.gain_hi) || !(nz.quant_step >= 0.f) ||
        !(nz.radius_rho >= 0.f) || !(nz.drift_sigma >= 0.f) || !(nz.white_sigma >= 0.f))
      return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "bad noise parameter range");
    if (nz.xtalk_kind == 2 && !(nz.xtalk_sigma > 0.f))
      return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "dense crosstalk needs sigma > 0");
  }
  const uint32_t om = cfg->output_mask;
  if ((om & TG_OUT_NOISY) && !noise) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "noisy outputs need noise");

  tg_readout* h = new (std::nothrow) tg_readout();
  if (!h) return fail(nullptr, TG_ERR_OUT_OF_MEMORY, "host allocation");
  h->cfg = *cfg;
  h->E = E; h->L = L; h->T = T; h->n_obj = NO; h->W = (T + 63) / 64;
  h->noise = noise;
  h->xt = noise ? nz.xtalk_kind : 0;
  h->hy = noise ? nz.hyst_mode : 0;
  int64_t total_vals = 0;
  for (int g = 0; g < NO; ++g) total_vals += (int64_t)cfg->grids[g].n * cfg->grids[g].n * cfg->grids[g].n;

  // host staging
  std::vector<float4> tA(T), tB(T);
  std::vector<int32_t> link_of(T);
  for (int l = 0; l < L; ++l)
    for (int j = off[l]; j < off[l + 1]; ++j) link_of[j] = l;
  for (int j = 0; j < T; ++j) {
    tA[j] = make_float4(cfg->taxel_pos[3 * j], cfg->taxel_pos[3 * j + 1], cfg->taxel_pos[3 * j + 2], cfg->taxel_radius[j]);
    int32_t lk = link_of[j];
    float lkf;
    memcpy(&lkf, &lk, 4);
    tB[j] = make_float4(cfg->taxel_normal[3 * j], cfg->taxel_normal[3 * j + 1], cfg->taxel_normal[3 * j + 2], lkf);
  }
  std::vector<GridDesc> gd(NO);
  int64_t goff = 0;
  for (int g = 0; g < NO; ++g) {
    const tg_sdf_grid& G = cfg->grids[g];
    for (int i = 0; i < 3; ++i) gd[g].origin[i] = G.origin[i];
    gd[g].spacing = G.spacing;
    volatile float one = 1.0f;
    gd[g].hinv = one / G.spacing;
    gd[g].nm1 = (float)(G.n - 1);
    gd[g].n = G.n;
    gd[g].pad = 0;
    gd[g].offset = goff;
    goff += (int64_t)G.n * G.n * G.n;
  }

  KParams& k = h->kp;
  hipError_t e = hipSuccess;
  float4 *dA = nullptr, *dB = nullptr;
  int32_t* dOff = nullptr;
  GridDesc* dG = nullptr;
  float* dV = nullptr;
  const int64_t ET = (int64_t)E * T;
  if ((e = dalloc(h, &dA, T)) != hipSuccess || (e = dalloc(h, &dB, T)) != hipSuccess ||
      (e = dalloc(h, &dOff, L + 1)) != hipSuccess || (e = dalloc(h, &dG, NO)) != hipSuccess ||
      (e = dalloc(h, &dV, total_vals)) != hipSuccess) {
    tg_readout_destroy(h);
    return fail(nullptr, TG_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  float *dDrift = nullptr, *dHy = nullptr, *dHp = nullptr, *dStuck = nullptr, *dGain = nullptr;
  uint8_t *dSch = nullptr, *dDead = nullptr;
  if ((e = dalloc(h, &dDrift, 6 * ET)) != hipSuccess || (e = dalloc(h, &dHy, 6 * ET)) != hipSuccess ||
      (e = dalloc(h, &dHp, 6 * ET)) != hipSuccess || (e = dalloc(h, &dStuck, ET)) != hipSuccess ||
      (e = dalloc(h, &dGain, ET)) != hipSuccess || (e = dalloc(h, &dSch, ET)) != hipSuccess ||
      (e = dalloc(h, &dDead, ET)) != hipSuccess) {
    tg_readout_destroy(h);
    return fail(nullptr, TG_ERR_OUT_OF_MEMORY, std::string("hipMalloc (state): ") + hipGetErrorString(e));
  }
  h->state_bytes = (size_t)ET * (6 * 3 * 4 + 4 + 4 + 1 + 1);
  e = hipMemcpy(dA, tA.data(), T * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dB, tB.data(), T * sizeof(float4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dOff, off, (L + 1) * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dG, gd.data(), NO * sizeof(GridDesc), hipMemcpyHostToDevice);
  for (int g = 0; g < NO && e == hipSuccess; ++g) {
    const tg_sdf_grid& G = cfg->grids[g];
    e = hipMemcpy(dV + gd[g].offset, G.values, (size_t)G.n * G.n * G.n * sizeof(float), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    tg_readout_destroy(h);
    return fail(nullptr, TG_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }

  k.E = E; k.L = L; k.T = T; k.n_obj = NO; k.W = h->W;
  k.taxA = dA; k.taxB = dB; k.link_off = dOff; k.grids = dG; k.grid_vals = dV;
  k.k_n = cfg->k_n; k.c_n = cfg->c_n; k.alpha = cfg->alpha; k.nk_t = -cfg->k_t; k.k_w = cfg->k_w; k.mu = cfg->mu;
  k.Rp = cfg->prox_range;
  {
    volatile float one = 1.0f;
    k.rpinv = one / cfg->prox_range;
  }
  k.eta_on = cfg->eta_on;
  k.eta_off = noise ? nz.eta_off : cfg->eta_on;
  k.alpha_is_one = cfg->alpha == 1.0f;
  k.spring_only = cfg->ft_spring_only != 0;
  k.key0 = (uint32_t)nz.seed;
  k.key1 = (uint32_t)(nz.seed >> 32);
  k.drift_sigma = noise ? nz.drift_sigma : 0.f;
  k.white_sigma = noise ? nz.white_sigma : 0.f;
  k.bias = noise ? nz.bias : 0.f;
  k.quant = noise ? nz.quant_step : 0.f;
  {
    volatile float one = 1.0f;
    k.qinv = (noise && nz.quant_step > 0.f) ? one / nz.quant_step : 0.f;
    k.kload = nz.tau_load_steps > 0.f ? one / nz.tau_load_steps : 1.f;
    k.kunload = nz.tau_unload_steps > 0.f ? one / nz.tau_unload_steps : 1.f;
  }
  k.decay = (nz.maxwell_tau_s > 0.f) ? (float)std::exp(-(double)nz.dt_s / (double)nz.maxwell_tau_s) : 0.f;
  k.beta = nz.maxwell_beta;
  k.two_rho = 2.0f * nz.radius_rho;
  k.neg_rho = -nz.radius_rho;
  k.chi = nz.xtalk_chi;
  k.has_gain = noise && !(nz.gain_lo == 1.0f && nz.gain_hi == 1.0f);
  k.has_stuck = noise && nz.p_dead > 0.f;
  k.has_radius = noise && nz.radius_rho > 0.f;
  k.drift = dDrift; k.hyst = dHy; k.hyst_prev = dHp; k.schmitt = dSch; k.dead = dDead; k.stuck = dStuck;
  k.gain = dGain;
  h->stuck_lo = nz.stuck_lo;
  h->stuck_span = nz.stuck_hi - nz.stuck_lo;
  h->gain_lo = noise ? nz.gain_lo : 1.f;
  h->gain_span = noise ? nz.gain_hi - nz.gain_lo : 0.f;
  {
    double thr = std::floor((double)(noise ? nz.p_dead : 0.f) * 4294967296.0);
    h->dead_thr = (unsigned long long)std::min(thr, 4294967296.0);
  }

  // launch shape: whole envs per block, at most 1024 threads
  h->eb = std::max(1, std::min(E, 1024 / T));
  h->threads = ((h->eb * T + 63) / 64) * 64;
  k.eb = h->eb;
  k.tpad = 0;
  if (h->xt == 2) {
    tg_status st = xt_dense_setup(h->xtd, cfg, h->eb, &h->err);
    if (st != TG_OK) {
      std::string m = h->err;
      tg_readout_destroy(h);
      return fail(nullptr, st, m);
    }
    k.xt_afrag = h->xtd.afrag; k.xt_items = h->xtd.items; k.xt_n_items = h->xtd.n_items;
    k.tpad = h->xtd.tpad; k.xt_poff = h->xtd.poff;
  }
  LdsLayout ll = lds_layout(h->eb, L, T, h->W, noise, h->xt, k.tpad);
  h->lds = ll.total;
  if (h->lds > 160 * 1024) {
    tg_readout_destroy(h);
    return fail(nullptr, TG_ERR_UNSUPPORTED, "LDS footprint exceeds 160 KiB");
  }
  KernelFn kf = select_kernel(noise, h->xt, h->hy, 0);
  KernelFn kf1 = select_kernel(noise, h->xt, h->hy, 1);
  if (!kf || !kf1) {
    tg_readout_destroy(h);
    return fail(nullptr, TG_ERR_UNSUPPORTED, "no kernel for this noise configuration");
  }
  e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)kf1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds);
  if (e != hipSuccess) {
    tg_readout_destroy(h);
    return fail(nullptr, TG_ERR_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  }
  tg_status st = tg_readout_reset(h, nullptr, 0, nullptr);
  if (st == TG_OK) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) st = TG_ERR_HIP;
  }
  if (st != TG_OK) {
    std::string m = h->err;
    tg_readout_destroy(h);
    return fail(nullptr, st, "initial reset failed: " + m);
  }
  *out = h;
  return TG_OK;
}

tg_status tg_readout_reset(tg_readout* h, const uint8_t* env_mask_dev, int64_t step, void* hip_stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->err.clear();
  if (step < 0 || step >= (int64_t(1) << 32)) return fail(h, TG_ERR_INVALID_ARGUMENT, "step out of [0, 2^32)");
  const int64_t ET = (int64_t)h->E * h->T;
  const int threads = 256;
  const int blocks = (int)((ET + threads - 1) / threads);
  hipLaunchKernelGGL(tg_reset_kernel, dim3(blocks), dim3(threads), 0, (hipStream_t)hip_stream, h->kp, env_mask_dev,
                     step, h->stuck_lo, h->stuck_span, h->gain_lo, h->gain_span, h->dead_thr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(h, TG_ERR_HIP, std::string("reset launch: ") + hipGetErrorString(e));
  return TG_OK;
}

tg_status tg_readout_rollout(tg_readout* h, const tg_step_inputs* in, const tg_step_outputs* out, int32_t n_steps,
                             void* hip_stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->err.clear();
  if (!in || !out) return fail(h, TG_ERR_INVALID_ARGUMENT, "inputs/outputs struct is NULL");
  if (n_steps < 0) return fail(h, TG_ERR_INVALID_ARGUMENT, "n_steps < 0");
  if (n_steps == 0) return TG_OK;
  if (in->step < 0 || in->step + n_steps > (int64_t(1) << 32))
    return fail(h, TG_ERR_INVALID_ARGUMENT, "steps must lie in [0, 2^32)");
  if (!in->link_state || !in->obj_id) return fail(h, TG_ERR_INVALID_ARGUMENT, "link_state and obj_id are required");
  if (!aligned(in->link_state, 16) || !aligned(in->obj_id, 16) || (in->obj_state && !aligned(in->obj_state, 16)))
    return fail(h, TG_ERR_INVALID_ARGUMENT, "input pointers must be 16-byte aligned");
  const uint32_t om = h->cfg.output_mask;
  struct Req { const void* p; uint32_t bit; const char* name; } req[] = {
      {out->contact_bits, TG_OUT_BITS, "contact_bits"},     {out->depth, TG_OUT_DEPTH, "depth"},
      {out->prox, TG_OUT_PROX, "prox"},                     {out->ft, TG_OUT_FT, "ft"},
      {out->ft_noisy, TG_OUT_NOISY, "ft_noisy"},            {out->contact_bits_noisy, TG_OUT_NOISY, "contact_bits_noisy"},
      {out->normal, TG_OUT_NORMAL, "normal"},               {out->surfdist, TG_OUT_SURFDIST, "surfdist"},
      {out->link_sums, TG_OUT_LINK_SUMS, "link_sums"}};
  for (const Req& r : req) {
    const bool want = (om & r.bit) != 0;
    if (want && !r.p) return fail(h, TG_ERR_INVALID_ARGUMENT, std::string(r.name) + " requested but NULL");
    if (!want && r.p) return fail(h, TG_ERR_INVALID_ARGUMENT, std::string(r.name) + " not requested but non-NULL");
    if (r.p && !aligned(r.p, 16)) return fail(h, TG_ERR_INVALID_ARGUMENT, std::string(r.name) + " misaligned");
  }
  const bool want_ln = (om & TG_OUT_LINK_SUMS) && (om & TG_OUT_NOISY);
  if (want_ln != (out->link_sums_noisy != nullptr))
    return fail(h, TG_ERR_INVALID_ARGUMENT, "link_sums_noisy must be set iff LINK_SUMS and NOISY are requested");
  if (out->link_sums_noisy && !aligned(out->link_sums_noisy, 16))
    return fail(h, TG_ERR_INVALID_ARGUMENT, "link_sums_noisy misaligned");

  KParams k = h->kp;
  k.n_steps = n_steps;
  k.step0 = in->step;
  k.link_state = in->link_state;
  k.obj_state = in->obj_state;
  k.obj_id = in->obj_id;
  k.bits = (unsigned long long*)out->contact_bits;
  k.bits_noisy = (unsigned long long*)out->contact_bits_noisy;
  k.depth = out->depth; k.prox = out->prox; k.surfdist = out->surfdist; k.ft = out->ft; k.ft_noisy = out->ft_noisy;
  k.normal = out->normal; k.link_sums = out->link_sums; k.link_sums_noisy = out->link_sums_noisy;
  KernelFn kf = select_kernel(h->noise, h->xt, h->hy, in->obj_state ? 1 : 0);
  const int blocks = (h->E + h->eb - 1) / h->eb;
  hipLaunchKernelGGL(kf, dim3(blocks), dim3(h->threads), h->lds, (hipStream_t)hip_stream, k);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(h, TG_ERR_HIP, std::string("readout launch: ") + hipGetErrorString(e));
  return TG_OK;
}

tg_status tg_readout_step(tg_readout* h, const tg_step_inputs* in, const tg_step_outputs* out, void* hip_stream) {
  return tg_readout_rollout(h, in, out, 1, hip_stream);
}

tg_status tg_readout_state_size(const tg_readout* h, size_t* bytes) {
  if (!h || !bytes) return TG_ERR_INVALID_ARGUMENT;
  *bytes = h->state_bytes;
  return TG_OK;
}

static tg_status copy_state(tg_readout* h, void* buf, size_t bytes, bool to_buf, void* stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->err.clear();
  if (!buf || bytes != h->state_bytes) return fail(h, TG_ERR_INVALID_ARGUMENT, "state buffer size mismatch");
  const size_t ET = (size_t)h->E * h->T;
  struct Part { void* p; size_t n; } parts[] = {
      {h->kp.drift, 6 * ET * 4}, {h->kp.hyst, 6 * ET * 4}, {h->kp.hyst_prev, 6 * ET * 4},
      {h->kp.stuck, ET * 4},     {h->kp.gain, ET * 4},     {h->kp.schmitt, ET},
      {h->kp.dead, ET}};
  size_t off = 0;
  for (const Part& pt : parts) {
    char* b = (char*)buf + off;
    hipError_t e = to_buf ? hipMemcpyAsync(b, pt.p, pt.n, hipMemcpyDeviceToDevice, (hipStream_t)stream)
                          : hipMemcpyAsync(pt.p, b, pt.n, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return fail(h, TG_ERR_HIP, std::string("state copy: ") + hipGetErrorString(e));
    off += pt.n;
  }
  return TG_OK;
}

tg_status tg_readout_get_state(tg_readout* h, void* dst_dev, size_t bytes, void* hip_stream) {
  return copy_state(h, dst_dev, bytes, true, hip_stream);
}
tg_status tg_readout_set_state(tg_readout* h, const void* src_dev, size_t bytes, void* hip_stream) {
  return copy_state(h, const_cast<void*>(src_dev), bytes, false, hip_stream);
}

tg_status tg_readout_launch_shape(const tg_readout* h, int32_t* envs_per_block, int32_t* threads) {
  if (!h || !envs_per_block || !threads) return TG_ERR_INVALID_ARGUMENT;
  *envs_per_block = h->eb;
  *threads = h->threads;
  return TG_OK;
}

}  // extern "C"
