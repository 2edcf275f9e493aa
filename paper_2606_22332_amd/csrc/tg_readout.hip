// C-ABI implementation of the tactile readout library (include/tg_readout.h) and the
// kernel entry points.  Build: hipcc --offload-arch=gfx950 -O3 -ffp-contract=off
//   -fno-gpu-flush-denormals-to-zero -fhip-fp32-correctly-rounded-divide-sqrt -shared -fPIC
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tg_readout.h"
#include "link_kernel.h"
#include "neural_kernel.h"
#include "thermal_kernel.h"
#include "nsdf_host.h"

using namespace tg;

namespace {

thread_local std::string g_create_error;

inline int32_t align16i(int64_t x) { return (int32_t)((x + 15) & ~int64_t(15)); }

// Values of an n^3 grid in 4 x 4 x 4 bricks (the layout GridDesc describes), zero padded.
inline int64_t brick_values(int n) {
  const int64_t nb = (n + 3) / 4;
  return nb * nb * nb * 64;
}
void to_bricks(const float* v, int n, float* out) {
  const int nb = (n + 3) / 4;
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const int64_t b = ((int64_t)(z >> 2) * nb + (y >> 2)) * nb + (x >> 2);
        out[b * 64 + ((z & 3) * 4 + (y & 3)) * 4 + (x & 3)] = v[((int64_t)z * n + y) * n + x];
      }
}

}  // namespace

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

// Clear the contact-bit words of a rollout (one or two planes of n words) before the readout
// kernel ors its bits into them.  A kernel rather than a memset, so that a captured rollout
// holds no memset node.
__global__ void tg_clear_words_kernel(unsigned long long* a, unsigned long long* b, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (a) a[i] = 0ull;
    if (b) b[i] = 0ull;
  }
}

// Links without taxels get no work item; their per-link sums are zero (no force, no contact), so
// their columns of the [S][11][L][E] sums are cleared before the launch.
__global__ void tg_clear_empty_link_sums_kernel(float* a, float* b, const int32_t* empty, int n_empty, int64_t E,
                                                int64_t L, int64_t total) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t e = i % E, r = i / E;
    const int64_t m = r % n_empty, sc = r / n_empty;   // sc = step * 11 + channel
    const int64_t o = sc * L * E + (int64_t)empty[m] * E + e;
    if (a) a[o] = 0.f;
    if (b) b[o] = 0.f;
  }
}

// ------------------------------------------------------------------------------------------------
// handle
// ------------------------------------------------------------------------------------------------
struct tg_readout {
  tg_readout_config cfg{};
  int E = 0, L = 0, T = 0, n_obj = 0, W = 0;
  int threads = 64, target = 512;
  size_t lds = 0;
  std::vector<LinkInfo> links;
  LinkInfo* d_links = nullptr;
  int2* d_items = nullptr;
  int32_t* d_empty = nullptr;   // links without taxels
  int n_empty = 0;
  uint32_t* d_err = nullptr;    // device error word (KParams::err)
  int xt = 0, hy = 0, noise = 0, full = 1;
  uint64_t cfg_hash = 0;   // what the autotuner's plan depends on (sizes, link layout, kernel variant)
  KParams kp{};
  KParams* d_kp = nullptr;   // device copy read by the kernels
  std::vector<void*> allocs;
  std::string err;
  float stuck_lo = 0, stuck_span = 0, gain_lo = 1, gain_span = 0;
  unsigned long long dead_thr = 0;
  size_t state_bytes = 0;
  XtDense xtd;
  // neural SDF backend (sdf_mode 1)
  int neural = 0;
  NBox* d_boxes = nullptr;
  uint32_t* d_img = nullptr;
  int32_t* d_order = nullptr;
  uint16_t* d_silu = nullptr;
  size_t neural_lds = 0;
  // launch graph of the rollout (recorded on a private stream, replayed on the caller's)
  int graph_on = 1;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  // thermal fields
  int thermal = 0;
  ThermalParams thp{};
  ThermalParams* d_thp = nullptr;
  size_t field_bytes = 0;
  size_t tmeas_bytes = 0;     // measured readings behind the sensor lag (spectral solver)
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

using KernelFn = void (*)(const KLaunch);

template <int N, int X, int Y, int O, int F>
KernelFn pick() { return tg_link_kernel<N, X, Y, O, F>; }

template <int F>
KernelFn select_kernel_f(int noise, int xt, int hy, int obj) {
  if (!noise) return obj ? pick<0, 0, 0, 1, F>() : pick<0, 0, 0, 0, F>();
#define TG_PICK(X, Y)                                                   \
  if (xt == X && hy == Y) return obj ? pick<1, X, Y, 1, F>() : pick<1, X, Y, 0, F>();
  TG_PICK(0, 0) TG_PICK(0, 1) TG_PICK(0, 2)
  TG_PICK(1, 0) TG_PICK(1, 1) TG_PICK(1, 2)
  TG_PICK(2, 0) TG_PICK(2, 1) TG_PICK(2, 2)
  TG_PICK(3, 0) TG_PICK(3, 1) TG_PICK(3, 2)
#undef TG_PICK
  return nullptr;
}

// Crosstalk variant of the readout kernel: the dense kind reads its A fragments from LDS when
// the plan staged them, else from L2.
int kernel_xt(const tg_readout* h) { return h->xt == 2 && !h->kp.afr_lds ? 3 : h->xt; }

KernelFn select_kernel(int noise, int xt, int hy, int obj, int full) {
  return full ? select_kernel_f<1>(noise, xt, hy, obj) : select_kernel_f<0>(noise, xt, hy, obj);
}

// Work plan: envs per block for each link (about `target` readouts per block), the
// (link, first env) items sorted by env, the LDS carve-up sized for the largest link.
tg_status plan_links(tg_readout* h, int target) {
  const int L = h->L, E = h->E;
  const int32_t* off = h->cfg.link_taxel_offset;
  int nthr = 64;
  for (int l = 0; l < L; ++l) {
    LinkInfo& li = h->links[l];
    li.off = off[l];
    li.n = off[l + 1] - off[l];
    if (li.n > 512) return TG_ERR_UNSUPPORTED;
    // envs per block: ~target readouts, at most 36 envs so that the 14 prefetched scalars per env
    // fit one per lane
    li.np = li.n > 0 ? (li.n + 7) & ~7 : 8;   // lanes per env: whole 8-lane groups
    li.envs = std::max(1, std::min(std::min(E, 36), target / li.np));
    li.nwin = li.n > 0 ? ((li.off + li.n - 1) >> 6) - (li.off >> 6) + 1 : 1;
    li.nt = (6 * li.envs + 15) / 16;
    const int n16 = ((li.n + 15) / 16) * 16, n32 = ((li.n + 31) / 32) * 32;
    li.kp = n32 + 8;    // B staging column stride (bf16): K tiles of 32, 16-byte aligned columns
    li.kpd = n16 + 4;   // result staging row stride (floats)
    nthr = std::max(nthr, ((li.envs * li.np + 63) / 64) * 64);
  }
  {  // the per-step input prefetch parks 14 scalars per env, one per lane
    int max_envs = 1;
    for (int l = 0; l < L; ++l) max_envs = std::max(max_envs, h->links[l].envs);
    nthr = std::max(nthr, ((14 * max_envs + 63) / 64) * 64);
  }
  if (nthr > 512) return TG_ERR_UNSUPPORTED;
  for (int l = 0; l < L; ++l)   // the per-step epilogues take one pass: one lane per item
    if (10 * h->links[l].envs > nthr || h->links[l].envs * h->links[l].nwin > nthr) return TG_ERR_UNSUPPORTED;
  h->threads = nthr;
  // LDS layout: max over links of each region
  int64_t pose = 0, bits = 0, bt = 0, dt = 0, tax = 0;
  for (int l = 0; l < L; ++l) {
    const LinkInfo& li = h->links[l];
    pose = std::max<int64_t>(pose, li.envs);
    bits = std::max<int64_t>(bits, (int64_t)li.envs * li.nwin * 2);
    tax = std::max<int64_t>(tax, (int64_t)li.n * 32);
    if (h->xt == 2) {
      bt = std::max<int64_t>(bt, (int64_t)li.nt * 16 * li.kp * 2);
      dt = std::max<int64_t>(dt, (int64_t)6 * li.envs * li.kpd * 4);
    }
  }
  LinkLds& d = h->kp.lds;
  int64_t o = 0;
  d.pose = (int32_t)o; o = align16i(o + 2 * pose * (int64_t)sizeof(Pose));
  d.opose = (int32_t)o; o = align16i(o + 2 * pose * (int64_t)sizeof(Pose));
  d.oid = (int32_t)o; o = align16i(o + 2 * pose * 4);
  d.bits = (int32_t)o; o = align16i(o + 2 * 2 * bits * 4);
  d.sums = (int32_t)o; o = align16i(o + 10 * (int64_t)(nthr / 8 + 1) * 4);   // channel stride groups + 1
  d.xz = (int32_t)o; o = align16i(o + (h->xt == 1 ? 6 * (int64_t)nthr * 4 : 0));
  d.tax = (int32_t)o; o = align16i(o + tax);
  h->kp.gtab_lds = h->n_obj <= 256;
  d.gtab = (int32_t)o; o = align16i(o + (h->kp.gtab_lds ? (int64_t)h->n_obj * (int64_t)sizeof(GridDesc) : 0));
  d.raw = (int32_t)o; o = align16i(o + 2 * 14 * pose * 4);
  d.bt = (int32_t)o; o = align16i(o + bt);
  d.dt = (int32_t)o; o = align16i(o + dt);
  // the dense crosstalk A fragments of the largest link, resident in LDS when they fit
  int64_t afr = 0;
  if (h->xt == 2)
    for (int l = 0; l < L; ++l) afr = std::max<int64_t>(afr, (int64_t)h->links[l].mt * h->links[l].kt * 64 * 16);
  // stage them only when the CU still holds the 16 waves its VGPR budget allows (128 per lane)
  const int64_t blocks_wanted = std::max(1, 16 / (nthr / 64));
  h->kp.afr_lds = (h->xt == 2 && afr > 0 && align16i(o + afr) * blocks_wanted <= 160 * 1024) ? 1 : 0;
  d.afr = (int32_t)o; o = align16i(o + (h->kp.afr_lds ? afr : 0));
  d.total = (int32_t)o;
  h->lds = (size_t)o;
  // items, env-major so that neighbouring blocks share envs (and objects)
  std::vector<int2> items;
  std::vector<int> next(L, 0);
  for (int e0 = 0; e0 < E; ++e0)
    for (int l = 0; l < L; ++l)
      if (h->links[l].n > 0 && e0 == next[l]) {
        items.push_back(make_int2(l, e0));
        next[l] += h->links[l].envs;
      }
  h->kp.n_items = (int32_t)items.size();
  h->kp.n_items_pad = (int32_t)(((items.size() + 7) / 8) * 8);
  if (h->d_items) { (void)hipFree(h->d_items); h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), (void*)h->d_items)); }
  if (h->d_links) { (void)hipFree(h->d_links); h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), (void*)h->d_links)); }
  h->d_items = nullptr;
  h->d_links = nullptr;
  hipError_t e = dalloc(h, &h->d_items, items.size());
  if (e == hipSuccess) e = dalloc(h, &h->d_links, L);
  if (e == hipSuccess) e = hipMemcpy(h->d_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_links, h->links.data(), L * sizeof(LinkInfo), hipMemcpyHostToDevice);
  if (e != hipSuccess) return TG_ERR_HIP;
  h->kp.items = h->d_items;
  h->kp.links = h->d_links;
  h->target = target;
  return TG_OK;
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
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->cap) (void)hipStreamDestroy(h->cap);
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
  if ((int64_t)E * T * 4 > (int64_t)0xffffffffLL)
    return fail(nullptr, TG_ERR_UNSUPPORTED, "num_envs * num_taxels * 4 must fit 32 bits (shard the envs)");
  if ((int64_t)E * L * 11 * 4 > (int64_t)0xffffffffLL)
    return fail(nullptr, TG_ERR_UNSUPPORTED, "num_envs * num_links * 44 must fit 32 bits (shard the envs)");
  if (cfg->sdf_mode != 0 && cfg->sdf_mode != 1) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "sdf_mode must be 0 or 1");
  if (cfg->sdf_mode == 1) {
    if (noise) return fail(nullptr, TG_ERR_UNSUPPORTED, "the neural SDF backend computes the clean readout only");
    if (!cfg->nsdf_params) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "sdf_mode 1 needs nsdf_params");
    if (!(cfg->nsdf_band >= 0.f)) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "nsdf_band must be >= 0");
    if (neural_lds_bytes(L) + nsdf::SILU_BYTES > 160 * 1024) return fail(nullptr, TG_ERR_UNSUPPORTED, "too many links for the neural kernel");
  }
  std::vector<int32_t> taxel_vox;
  double th_r = 0, th_g = 0, th_rf = 0, th_kap = 0;
  if (cfg->thermal) {
    const tg_thermal_desc& td = *cfg->thermal;
    if (cfg->sdf_mode != 0) return fail(nullptr, TG_ERR_UNSUPPORTED, "thermal fields need the grid SDF backend");
    if (td.n != TH_N) return fail(nullptr, TG_ERR_UNSUPPORTED, "thermal fields must have 16 voxels per axis");
    if (td.num_fields < 1 || !td.field_links || !td.T_obj)
      return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "thermal: need fields, links and object temperatures");
    if (!(td.dx > 0.f) || !(td.dt > 0.f) || !(td.k_sensor > 0.f) || !(td.rho_cp > 0.f) || !(td.k_object > 0.f) ||
        !(td.emissivity >= 0.f) || !(td.d_w >= 0.f) || !(td.P_gen >= 0.f))
      return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "thermal: bad material constants");
    taxel_vox.assign(T, -1);
    std::vector<int> per_vox;
    int m_max = 0;
    for (int f = 0; f < td.num_fields; ++f) {
      const int l = td.field_links[f];
      if (l < 0 || l >= L) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "thermal: field link out of range");
      for (int f2 = 0; f2 < f; ++f2)
        if (td.field_links[f2] == l) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "thermal: duplicate field link");
      if (off[l + 1] - off[l] > 512) return fail(nullptr, TG_ERR_UNSUPPORTED, "thermal link with more than 512 taxels");
      per_vox.assign(TH_N * TH_N, 0);
      for (int j = off[l]; j < off[l + 1]; ++j) {
        int idx[2];
        for (int d = 0; d < 2; ++d) {
          int i = (int)std::floor(((double)cfg->taxel_pos[3 * j + d] - (double)td.origin[d]) / (double)td.dx);
          idx[d] = i < 0 ? 0 : (i > TH_N - 1 ? TH_N - 1 : i);
        }
        taxel_vox[j] = idx[1] * TH_N + idx[0];
        m_max = std::max(m_max, ++per_vox[taxel_vox[j]]);
      }
    }
    // derived constants (FP64, rounded once to FP32 for the kernel)
    const double dx = td.dx, rc = td.rho_cp, dt = td.dt, Ta = (double)td.T_amb + 273.15;
    const double alpha = (double)td.k_sensor / rc;
    const double h_r = 4.0 * (double)td.emissivity * 5.670374419e-8 * Ta * Ta * Ta;
    const double k_eff = 2.0 * (double)td.k_sensor * (double)td.k_object / ((double)td.k_sensor + (double)td.k_object);
    th_r = alpha * dt / (dx * dx);
    th_rf = dt * h_r / (rc * dx);
    th_g = dt * (double)td.P_gen / ((double)TH_N * TH_N * TH_N * rc * dx * dx * dx);
    th_kap = dt * 3.14159265358979323846 * (double)td.d_w * k_eff / (rc * dx * dx * dx);
    // largest clean depth the grids allow: max R_j + max over objects of -min(phi)
    double rmax = 0, dmin = 0;
    for (int j = 0; j < T; ++j) rmax = std::max(rmax, (double)cfg->taxel_radius[j]);
    for (int g = 0; g < NO; ++g) {
      const tg_sdf_grid& G = cfg->grids[g];
      const int64_t nv = (int64_t)G.n * G.n * G.n;
      for (int64_t i = 0; i < nv; ++i) dmin = std::min(dmin, (double)G.values[i]);
    }
    if (td.solver == 1) {
      if (!(td.h_conv >= 0.f)) return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "thermal: negative h_conv");
      const double TaM = Ta + 100.0;
      const double lin = 3.0 * (4.0 * (double)td.emissivity * 5.670374419e-8 * TaM * TaM * TaM + (double)td.h_conv) *
                         dt / (rc * dx);
      if (!(th_kap * (rmax - dmin) * (double)m_max <= 1.0) || !(lin <= 1.0))
        return fail(nullptr, TG_ERR_UNSTABLE, "thermal step not stable: kappa d_max m or the surface loss > 1");
      if (td.lag_tau > 0.f)
        for (int f = 0; f < td.num_fields; ++f) {
          const int l = td.field_links[f];
          if (off[l + 1] - off[l] > TH_THREADS)
            return fail(nullptr, TG_ERR_UNSUPPORTED, "sensor lag on a thermal link of more than 256 taxels");
        }
    } else if (td.solver != 0) {
      return fail(nullptr, TG_ERR_INVALID_ARGUMENT, "thermal: solver must be 0 or 1");
    } else if (!(6.0 * th_r + 3.0 * th_rf + th_kap * (rmax - dmin) * (double)m_max <= 1.0)) {
      return fail(nullptr, TG_ERR_UNSTABLE, "thermal step not stable: 6 r + 3 rho_f + kappa d_max m > 1");
    }
  }

  tg_readout* h = new (std::nothrow) tg_readout();
  if (!h) return fail(nullptr, TG_ERR_OUT_OF_MEMORY, "host allocation");
  h->cfg = *cfg;
  h->E = E; h->L = L; h->T = T; h->n_obj = NO; h->W = (T + 63) / 64;
  h->noise = noise;
  h->xt = noise ? nz.xtalk_kind : 0;
  h->hy = noise ? nz.hyst_mode : 0;
  int64_t total_vals = 0;   // bricked: ceil(n/4)^3 bricks of 64 values per grid
  for (int g = 0; g < NO; ++g) total_vals += brick_values(cfg->grids[g].n);
  if (total_vals * 4 > (int64_t)0xffffffffLL) {   // grid corners are addressed with 32-bit byte offsets
    delete h;
    return fail(nullptr, TG_ERR_UNSUPPORTED, "grid values exceed 4 GiB");
  }

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
    gd[g].nb = (G.n + 3) / 4;
    gd[g].offset = goff;
    goff += brick_values(G.n);
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
  {
    std::vector<int32_t> empty;
    for (int l = 0; l < L; ++l)
      if (cfg->link_taxel_offset[l + 1] == cfg->link_taxel_offset[l]) empty.push_back(l);
    h->n_empty = (int)empty.size();
    if (h->n_empty > 0) {
      if ((e = dalloc(h, &h->d_empty, empty.size())) == hipSuccess)
        e = hipMemcpy(h->d_empty, empty.data(), empty.size() * sizeof(int32_t), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        tg_readout_destroy(h);
        return fail(nullptr, TG_ERR_OUT_OF_MEMORY, std::string("empty-link list: ") + hipGetErrorString(e));
      }
    }
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
    std::vector<float> bricks((size_t)brick_values(G.n), 0.f);
    to_bricks(G.values, G.n, bricks.data());
    e = hipMemcpy(dV + gd[g].offset, bricks.data(), bricks.size() * sizeof(float), hipMemcpyHostToDevice);
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

  // dense crosstalk blocks, then the work plan (links x env chunks)
  h->links.assign(L, LinkInfo{});
  if (h->xt == 2) {
    tg_status st = xt_dense_setup(h->xtd, cfg, h->links.data(), &h->err);
    if (st != TG_OK) {
      std::string m = h->err;
      tg_readout_destroy(h);
      return fail(nullptr, st, m);
    }
    k.xt_afrag = h->xtd.afrag;
  }
  {
    tg_status st = plan_links(h, 512);
    if (st != TG_OK) {
      tg_readout_destroy(h);
      return fail(nullptr, st, st == TG_ERR_UNSUPPORTED ? "a link has more than 512 taxels"
                                                        : "work plan upload failed");
    }
  }
  if (h->lds > 160 * 1024) {
    tg_readout_destroy(h);
    return fail(nullptr, TG_ERR_UNSUPPORTED, "LDS footprint exceeds 160 KiB");
  }
  e = dalloc(h, &h->d_err, 1);
  if (e == hipSuccess) e = hipMemset(h->d_err, 0, sizeof(uint32_t));
  h->kp.err = h->d_err;
  if (e == hipSuccess) e = dalloc(h, &h->d_kp, 1);
  if (e == hipSuccess) e = hipMemcpy(h->d_kp, &h->kp, sizeof(KParams), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    tg_readout_destroy(h);
    return fail(nullptr, TG_ERR_HIP, std::string("parameter upload: ") + hipGetErrorString(e));
  }
  h->full = (noise && (nz.white_sigma != 0.f || nz.bias != 0.f || nz.quant_step > 0.f || nz.radius_rho > 0.f ||
                        !(nz.gain_lo == 1.0f && nz.gain_hi == 1.0f))) ||
            (om & (TG_OUT_NORMAL | TG_OUT_SURFDIST)) != 0;
  {  // FNV-1a over what the fastest work plan depends on
    uint64_t x = 1469598103934665603ull;
    auto mix = [&x](int64_t v) {
      for (int b = 0; b < 8; ++b) {
        x ^= (uint64_t)((v >> (8 * b)) & 0xff);
        x *= 1099511628211ull;
      }
    };
    mix(E); mix(L); mix(T); mix(h->n_obj); mix(noise); mix(kernel_xt(h)); mix(h->hy); mix(h->full);
    mix(om); mix(cfg->sdf_mode); mix(cfg->thermal != nullptr);
    for (int l = 0; l <= L; ++l) mix(cfg->link_taxel_offset[l]);
    for (int o = 0; o < h->n_obj; ++o) mix(cfg->grids[o].n);
    h->cfg_hash = x;
  }
  KernelFn kf = select_kernel(noise, kernel_xt(h), h->hy, 0, h->full);
  KernelFn kf1 = select_kernel(noise, kernel_xt(h), h->hy, 1, h->full);
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
  if (cfg->sdf_mode == 1) {
    h->neural = 1;
    std::vector<NBox> bx(NO);
    for (int g = 0; g < NO; ++g) {
      const tg_sdf_grid& G = cfg->grids[g];
      const float ext = (float)(G.n - 1) * G.spacing;
      volatile float one = 1.0f;
      bx[g].half = 0.5f * ext;
      bx[g].half_inv = one / bx[g].half;
      for (int i = 0; i < 3; ++i) {
        bx[g].centre[i] = G.origin[i] + bx[g].half;
        bx[g].pad[i] = 0.f;
      }
    }
    e = dalloc(h, &h->d_boxes, NO);
    if (e == hipSuccess) e = dalloc(h, &h->d_img, (size_t)NO * nsdf::IMG_WORDS);
    if (e == hipSuccess) e = dalloc(h, &h->d_order, E);
    if (e == hipSuccess) e = dalloc(h, &h->d_silu, nsdf::SILU_ENTRIES);
    std::vector<uint16_t> silu(nsdf::SILU_ENTRIES);
    nsdf::build_silu_table(silu.data());
    if (e == hipSuccess) e = hipMemcpy(h->d_silu, silu.data(), nsdf::SILU_BYTES, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->d_boxes, bx.data(), NO * sizeof(NBox), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = nsdf_pack_images(cfg->nsdf_params, NO, h->d_img, nullptr);
    h->neural_lds = (size_t)neural_lds_bytes(L);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)tg_neural_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)h->neural_lds);
    if (e != hipSuccess) {
      tg_readout_destroy(h);
      return fail(nullptr, TG_ERR_HIP, std::string("neural SDF setup: ") + hipGetErrorString(e));
    }
  }
  if (cfg->thermal) {
    const tg_thermal_desc& td = *cfg->thermal;
    h->thermal = 1;
    ThermalParams& tp = h->thp;
    int32_t *dLinks = nullptr, *dVox = nullptr;
    float *dTobj = nullptr, *dF = nullptr;
    const int F = td.num_fields;
    h->field_bytes = (size_t)E * F * TH_N * TH_N * TH_N * sizeof(float);
    e = dalloc(h, &dLinks, F);
    if (e == hipSuccess) e = dalloc(h, &dVox, T);
    if (e == hipSuccess) e = dalloc(h, &dTobj, E);
    if (e == hipSuccess) e = dalloc(h, &dF, (size_t)E * F * TH_N * TH_N * TH_N);
    if (e == hipSuccess) e = dalloc(h, &h->d_thp, 1);
    if (e == hipSuccess) e = hipMemcpy(dLinks, td.field_links, F * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dVox, taxel_vox.data(), T * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dTobj, td.T_obj, E * sizeof(float), hipMemcpyHostToDevice);
    tp.F = F;
    tp.field_link = dLinks;
    tp.taxel_vox = dVox;
    tp.T_obj = dTobj;
    tp.fields = dF;
    tp.r = (float)th_r;
    tp.g = (float)th_g;
    tp.rho_f = (float)th_rf;
    tp.kappa = (float)th_kap;
    tp.T_amb = td.T_amb;
    tp.T0 = td.T0;
    tp.spectral = td.solver == 1;
    if (tp.spectral) {
      // orthonormal DCT-II of the 16 voxels of an axis, and the filter's correction per |m|^2
      std::vector<float> dct(TH_N * TH_N), hk(3 * (TH_N - 1) * (TH_N - 1) + 1);
      for (int m = 0; m < TH_N; ++m)
        for (int i = 0; i < TH_N; ++i)
          dct[m * TH_N + i] = (float)((m == 0 ? std::sqrt(1.0 / TH_N) : std::sqrt(2.0 / TH_N)) *
                                      std::cos(3.14159265358979323846 * m * (2 * i + 1) / (2.0 * TH_N)));
      const double a = (double)td.k_sensor / (double)td.rho_cp * (double)td.dt;
      const double kk = 3.14159265358979323846 / (TH_N * (double)td.dx);
      for (size_t q = 0; q < hk.size(); ++q) {
        const double k2 = std::max(kk * kk * (double)q, 1e-12);   // k^2 floored at eps = 1e-12
        hk[q] = (float)(a * k2 / (1.0 + a * k2));
      }
      float *dD = nullptr, *dH = nullptr;
      if (e == hipSuccess) e = dalloc(h, &dD, dct.size());
      if (e == hipSuccess) e = dalloc(h, &dH, hk.size());
      if (e == hipSuccess) e = hipMemcpy(dD, dct.data(), dct.size() * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(dH, hk.data(), hk.size() * 4, hipMemcpyHostToDevice);
      tp.dct = dD;
      tp.hk = dH;
      const double surf = (double)td.dt / ((double)td.rho_cp * (double)td.dx);
      tp.k_rad = (float)(surf * (double)td.emissivity * 5.670374419e-8);
      tp.k_conv = (float)(surf * (double)td.h_conv);
      tp.lag = td.lag_tau > 0.f ? (float)((double)td.dt / (double)td.lag_tau) : 0.f;
      if (tp.lag > 0.f) {
        float* dM = nullptr;
        if (e == hipSuccess) e = dalloc(h, &dM, (size_t)E * T);
        tp.t_meas = dM;
        h->tmeas_bytes = (size_t)E * T * sizeof(float);
      }
    }
    if (e == hipSuccess) e = hipMemcpy(h->d_thp, &tp, sizeof(ThermalParams), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      tg_readout_destroy(h);
      return fail(nullptr, TG_ERR_HIP, std::string("thermal setup: ") + hipGetErrorString(e));
    }
    h->state_bytes += h->field_bytes + h->tmeas_bytes;
  }
  e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    tg_readout_destroy(h);
    return fail(nullptr, TG_ERR_HIP, std::string("stream: ") + hipGetErrorString(e));
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
  if (h->thermal) {
    const int64_t nf = (int64_t)h->E * h->thp.F * TH_N * TH_N * TH_N;
    hipLaunchKernelGGL(tg_thermal_reset_kernel, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0,
                       (hipStream_t)hip_stream, (const ThermalParams*)h->d_thp, h->E, env_mask_dev);
    if (h->tmeas_bytes) {
      const int64_t nm = (int64_t)h->E * h->T;
      hipLaunchKernelGGL(tg_thermal_reset_meas_kernel, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0,
                         (hipStream_t)hip_stream, (const ThermalParams*)h->d_thp, h->E, h->T, env_mask_dev);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(h, TG_ERR_HIP, std::string("reset launch: ") + hipGetErrorString(e));
  return TG_OK;
}

static tg_status launch_rollout(tg_readout* h, const tg_step_inputs* in, const tg_step_outputs* out, int32_t n_steps,
                                hipStream_t stream);

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
      {out->link_sums, TG_OUT_LINK_SUMS, "link_sums"},     {out->temperature, TG_OUT_TEMP, "temperature"}};
  for (const Req& r : req) {
    const bool want = (om & r.bit) != 0;
    if (want && !r.p) return fail(h, TG_ERR_INVALID_ARGUMENT, std::string(r.name) + " requested but NULL");
    if (!want && r.p) return fail(h, TG_ERR_INVALID_ARGUMENT, std::string(r.name) + " not requested but non-NULL");
    if (r.p && !aligned(r.p, 16)) return fail(h, TG_ERR_INVALID_ARGUMENT, std::string(r.name) + " misaligned");
  }
  if ((om & TG_OUT_TEMP) && !h->thermal)
    return fail(h, TG_ERR_INVALID_ARGUMENT, "temperature requested without thermal fields");
  const bool want_ln = (om & TG_OUT_LINK_SUMS) && (om & TG_OUT_NOISY);
  if (want_ln != (out->link_sums_noisy != nullptr))
    return fail(h, TG_ERR_INVALID_ARGUMENT, "link_sums_noisy must be set iff LINK_SUMS and NOISY are requested");
  if (out->link_sums_noisy && !aligned(out->link_sums_noisy, 16))
    return fail(h, TG_ERR_INVALID_ARGUMENT, "link_sums_noisy misaligned");

  // Graph mode: record this call's launches on the private stream, then update the cached
  // executable graph (same kernels and shapes: only the arguments change) and replay it on the
  // caller's stream.  A caller that is itself capturing gets the plain launches.
  hipStream_t target = (hipStream_t)hip_stream;
  bool use_graph = h->graph_on != 0;
  if (use_graph) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(target, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) use_graph = false;
  }
  hipStream_t ls = use_graph ? h->cap : target;
  if (use_graph) {
    const hipError_t ce = hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal);
    if (ce != hipSuccess) return fail(h, TG_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
  }
  tg_status lst = launch_rollout(h, in, out, n_steps, ls);
  if (use_graph) {
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(ls, &g);
    if (ee != hipSuccess || lst != TG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return lst != TG_OK ? lst : fail(h, TG_ERR_HIP, std::string("graph capture end: ") + hipGetErrorString(ee));
    }
    if (h->gexec) {
      hipGraphNode_t en = nullptr;
      hipGraphExecUpdateResult ur;
      if (hipGraphExecUpdate(h->gexec, g, &en, &ur) != hipSuccess || ur != hipGraphExecUpdateSuccess) {
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
      }
    }
    hipError_t ge = hipSuccess;
    if (!h->gexec) ge = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ge == hipSuccess) ge = hipGraphLaunch(h->gexec, target);
    if (ge != hipSuccess) return fail(h, TG_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(ge));
    return TG_OK;
  }
  return lst;
}

static tg_status launch_rollout(tg_readout* h, const tg_step_inputs* in, const tg_step_outputs* out, int32_t n_steps,
                                hipStream_t stream) {
  void* hip_stream = (void*)stream;
  if (h->neural) {
    const int64_t EL = (int64_t)h->E * h->L, ET = (int64_t)h->E * h->T;
    hipStream_t st = (hipStream_t)hip_stream;
    for (int s = 0; s < n_steps; ++s) {
      hipLaunchKernelGGL(tg_group_kernel, dim3(1), dim3(1024), (h->n_obj + 2) * sizeof(int32_t), st,
                         in->obj_id + (int64_t)s * h->E, h->E, h->n_obj, h->d_order);
      NLaunch q{};
      q.kc = h->d_kp;
      q.boxes = h->d_boxes;
      q.images = h->d_img;
      q.silu = h->d_silu;
      q.order = h->d_order;
      q.band = h->cfg.nsdf_band;
      q.step = in->step + s;
      q.link_state = in->link_state + (int64_t)s * 13 * EL;
      q.obj_state = in->obj_state ? in->obj_state + (int64_t)s * 13 * h->E : nullptr;
      q.obj_id = in->obj_id + (int64_t)s * h->E;
      q.bits = out->contact_bits ? (unsigned long long*)out->contact_bits + (int64_t)s * h->E * h->W : nullptr;
      q.depth = out->depth ? out->depth + s * ET : nullptr;
      q.prox = out->prox ? out->prox + s * ET : nullptr;
      q.surfdist = out->surfdist ? out->surfdist + s * ET : nullptr;
      q.ft = out->ft ? out->ft + s * 6 * ET : nullptr;
      q.normal = out->normal ? out->normal + s * 3 * ET : nullptr;
      q.link_sums = out->link_sums ? out->link_sums + s * 11 * EL : nullptr;
      hipLaunchKernelGGL(tg_neural_kernel, dim3((h->E + NEU_ENVS - 1) / NEU_ENVS), dim3(NEU_THREADS), h->neural_lds,
                         st, q);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(h, TG_ERR_HIP, std::string("neural readout launch: ") + hipGetErrorString(e));
    return TG_OK;
  }

  KLaunch k{};
  k.kc = h->d_kp;
  k.n_steps = n_steps;
  k.step0 = in->step;
  k.link_state = in->link_state;
  k.obj_state = in->obj_state;
  k.obj_id = in->obj_id;
  k.bits = (unsigned long long*)out->contact_bits;
  k.bits_noisy = (unsigned long long*)out->contact_bits_noisy;
  k.depth = out->depth; k.prox = out->prox; k.surfdist = out->surfdist; k.ft = out->ft; k.ft_noisy = out->ft_noisy;
  k.normal = out->normal; k.link_sums = out->link_sums; k.link_sums_noisy = out->link_sums_noisy;
  KernelFn kf = select_kernel(h->noise, kernel_xt(h), h->hy, in->obj_state ? 1 : 0, h->full);
  if (k.bits || k.bits_noisy) {
    const int64_t nw = (int64_t)n_steps * h->E * h->W;
    const int64_t blocks = std::min<int64_t>((nw + 255) / 256, 16384);
    hipLaunchKernelGGL(tg_clear_words_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, k.bits,
                       k.bits_noisy, nw);
  }
  if (h->n_empty > 0 && (k.link_sums || k.link_sums_noisy)) {
    const int64_t total = (int64_t)n_steps * 11 * h->n_empty * h->E;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(tg_clear_empty_link_sums_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                       k.link_sums, k.link_sums_noisy, h->d_empty, h->n_empty, (int64_t)h->E, (int64_t)h->L, total);
  }
  hipLaunchKernelGGL(kf, dim3(h->kp.n_items_pad), dim3(h->threads), h->lds, (hipStream_t)hip_stream, k);
  if (h->thermal) {
    // After the readout, on the same stream: the fields take the depths the readout wrote (or
    // recompute them with its FP32 sequence when the rollout does not write depths).  Launched
    // beside it on a second stream instead, the thermal kernel measured slower (55 against 48.5 ms
    // at 4096 envs x 500 steps): the readout fills every wave slot of a CU, so the two only contend.
    ThermalLaunch t{};
    t.kc = h->d_kp;
    t.th = h->d_thp;
    t.n_steps = n_steps;
    t.link_state = in->link_state;
    t.obj_state = in->obj_state;
    t.obj_id = in->obj_id;
    t.temperature = out->temperature;
    t.depth = out->depth;   // null unless the rollout writes depths
    hipLaunchKernelGGL(h->thp.spectral ? tg_thermal_kernel<1> : tg_thermal_kernel<0>,
                       dim3((unsigned)(h->E * h->thp.F)), dim3(TH_THREADS), 0, (hipStream_t)hip_stream, t);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(h, TG_ERR_HIP, std::string("readout launch: ") + hipGetErrorString(e));
  return TG_OK;
}

tg_status tg_readout_step(tg_readout* h, const tg_step_inputs* in, const tg_step_outputs* out, void* hip_stream) {
  return tg_readout_rollout(h, in, out, 1, hip_stream);
}

tg_status tg_readout_set_graph(tg_readout* h, int32_t enable) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->graph_on = enable != 0;
  return TG_OK;
}

// Make `target` the handle's plan: link table, parameter block on the device, LDS attribute of
// both kernel variants; the captured rollout graph is dropped (its launch shape changed).
static tg_status apply_plan(tg_readout* h, int target) {
  tg_status ps = plan_links(h, target);
  if (ps == TG_OK && hipMemcpy(h->d_kp, &h->kp, sizeof(KParams), hipMemcpyHostToDevice) != hipSuccess) ps = TG_ERR_HIP;
  if (ps == TG_OK) {
    KernelFn kf = select_kernel(h->noise, kernel_xt(h), h->hy, 0, h->full);
    KernelFn kf1 = select_kernel(h->noise, kernel_xt(h), h->hy, 1, h->full);
    (void)hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds);
    (void)hipFuncSetAttribute((const void*)kf1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds);
  }
  if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
  return ps;
}

tg_status tg_readout_set_work_plan(tg_readout* h, int32_t readouts_per_workgroup) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->err.clear();
  if (h->neural) return TG_OK;
  if (readouts_per_workgroup < 64 || readouts_per_workgroup > 1024)
    return fail(h, TG_ERR_INVALID_ARGUMENT, "work plan: readouts per workgroup must be 64..1024");
  if (hipDeviceSynchronize() != hipSuccess) return fail(h, TG_ERR_HIP, "work plan: device synchronisation");
  const int prev = h->target;
  tg_status ps = plan_links(h, readouts_per_workgroup);
  if (ps == TG_OK && h->lds > 160 * 1024) {
    (void)apply_plan(h, prev);
    return fail(h, TG_ERR_INVALID_ARGUMENT, "work plan: LDS of this plan exceeds 160 KiB");
  }
  if (ps != TG_OK) {
    (void)apply_plan(h, prev);
    return fail(h, ps, "work plan: planning failed");
  }
  ps = apply_plan(h, readouts_per_workgroup);
  return ps == TG_OK ? TG_OK : fail(h, ps, "work plan: upload failed");
}

tg_status tg_readout_autotune(tg_readout* h, const tg_step_inputs* in, const tg_step_outputs* out, int32_t n_steps,
                              void* hip_stream, int32_t* best_target, float* best_ms) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->err.clear();
  if (n_steps < 1) return fail(h, TG_ERR_INVALID_ARGUMENT, "autotune needs n_steps >= 1");
  if (h->neural) {   // the neural kernel has no plan to tune
    if (best_target) *best_target = 0;
    if (best_ms) *best_ms = 0.f;
    return TG_OK;
  }
  // plans already tuned in this process for the same configuration and step count
  static std::mutex cache_mu;
  static std::map<uint64_t, std::pair<int, float>> cache;
  const uint64_t key = h->cfg_hash ^ ((uint64_t)n_steps * 0x9E3779B97F4A7C15ull) ^ (in && in->obj_state ? 1ull : 0ull);
  {
    std::lock_guard<std::mutex> lock(cache_mu);
    const auto it = cache.find(key);
    if (it != cache.end()) {
      const tg_status ps = apply_plan(h, it->second.first);
      if (ps != TG_OK) return fail(h, ps, "autotune: re-planning failed");
      if (best_target) *best_target = it->second.first;
      if (best_ms) *best_ms = it->second.second;
      return TG_OK;
    }
  }
  hipStream_t st = (hipStream_t)hip_stream;
  void* saved = nullptr;
  hipError_t e = hipMalloc(&saved, std::max<size_t>(h->state_bytes, 1));
  if (e != hipSuccess) return fail(h, TG_ERR_OUT_OF_MEMORY, "autotune: state buffer");
  tg_status rs = tg_readout_get_state(h, saved, h->state_bytes, hip_stream);
  hipEvent_t a = nullptr, b = nullptr;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  // readouts per workgroup; with one link per workgroup this sets both the envs per workgroup
  // and the waves per workgroup (about envs * n_l / 64 lanes' worth for each link)
  const int cand[] = {128, 192, 256, 320, 384, 448, 512};
  int best = h->target;
  float bms = 3.4e38f;
  for (int c : cand) {
    if (rs != TG_OK) break;
    if (hipStreamSynchronize(st) != hipSuccess) { rs = TG_ERR_HIP; break; }
    if (plan_links(h, c) != TG_OK || h->lds > 160 * 1024) continue;
    if (hipMemcpy(h->d_kp, &h->kp, sizeof(KParams), hipMemcpyHostToDevice) != hipSuccess) { rs = TG_ERR_HIP; break; }
    KernelFn kf = select_kernel(h->noise, kernel_xt(h), h->hy, in && in->obj_state ? 1 : 0, h->full);
    (void)hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds);
    if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
    rs = tg_readout_rollout(h, in, out, n_steps, hip_stream);           // warm-up
    float ms = 0.f;
    if (rs == TG_OK) {
      (void)hipEventRecord(a, st);
      rs = tg_readout_rollout(h, in, out, n_steps, hip_stream);
      (void)hipEventRecord(b, st);
      (void)hipEventSynchronize(b);
      (void)hipEventElapsedTime(&ms, a, b);
    }
    if (rs == TG_OK && std::getenv("TG_AUTOTUNE_VERBOSE"))
      std::fprintf(stderr, "tg_readout_autotune: %d readouts per workgroup, %d threads: %.3f ms\n", c, h->threads, ms);
    if (rs == TG_OK && ms < bms) { bms = ms; best = c; }
    if (rs == TG_OK) rs = tg_readout_set_state(h, saved, h->state_bytes, hip_stream);
  }
  (void)hipStreamSynchronize(st);
  tg_status ps = apply_plan(h, best);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(saved);
  if (rs != TG_OK) return rs;
  if (ps != TG_OK) return fail(h, ps, "autotune: re-planning failed");
  {
    std::lock_guard<std::mutex> lock(cache_mu);
    cache[key] = std::make_pair(best, bms);
  }
  if (best_target) *best_target = best;
  if (best_ms) *best_ms = bms;
  return TG_OK;
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
      {h->kp.dead, ET},          {h->thermal ? (void*)h->thp.fields : nullptr, h->field_bytes},
      {h->thermal ? (void*)h->thp.t_meas : nullptr, h->tmeas_bytes}};
  size_t off = 0;
  for (const Part& pt : parts) {
    if (!pt.p || pt.n == 0) continue;
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

static_assert(DEVERR_BAD_OBJECT_ID == TG_DEVERR_BAD_OBJECT_ID, "device error bits match the C header");

tg_status tg_readout_poll_errors(tg_readout* h, uint32_t* device_error_flags) {
  if (!h || !device_error_flags) return fail(h, TG_ERR_INVALID_ARGUMENT, "NULL handle or flags");
  uint32_t v = 0;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(&v, h->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(h->d_err, 0, sizeof(uint32_t));
  if (e != hipSuccess) return fail(h, TG_ERR_HIP, std::string("poll_errors: ") + hipGetErrorString(e));
  *device_error_flags = v;
  return TG_OK;
}

tg_status tg_readout_launch_shape(const tg_readout* h, int32_t* envs_per_block, int32_t* threads) {
  if (!h || !envs_per_block || !threads) return TG_ERR_INVALID_ARGUMENT;
  *envs_per_block = h->target;
  *threads = h->threads;
  return TG_OK;
}

}  // extern "C"
