// Contact-audio modal synthesis (App. E, contact audio) behind include/tg_audio.h.
//
// Work layout.  G lanes (1, 2, 4, 8 or 16) serve one (env, sensor link) pair and hold its bank's slots
// between them: MPL resonators per lane, states and coefficients in FP64 registers.  A wave holds
// 64 / G pairs and runs every step of the launch.  Per step:
//   1. excitation: the pair's lanes stride over the link's taxels, form f . m and
//      |f - (f . m) m| in FP64 and add them; DPP exchanges give every lane the totals;
//   2. scrape noise: the lanes share the block's Philox calls (four samples per call) and leave
//      xi[0..K) in the pair's LDS row;
//   3. the K samples, G at a time: each lane advances its resonators on u = g_scr F_t xi[k] (+ the
//      impact at k = 0) and forms its part of s[k] for the G samples; a transposed DPP reduction
//      (each exchange sends half of what a lane holds) leaves sample k0 + i in lane i of the pair,
//      which writes it, rounded to FP32, over xi[k0 + i] in the row;
//   4. the wave copies its rows, consecutive (env, link) blocks of the output, to HBM with
//      coalesced stores.
// Rows are padded to an odd length so the rows read at one sample index fall in distinct banks.
// Every row belongs to one wave (a workgroup is one wave), so barriers cost nothing.  The work is
// FP64 FMA issue: 3 FMAs per slot and sample (two for the recurrence, one for the output sum).
// G trades the cross-lane sums against the waves that hide the recurrence's latency (create's
// choice is explained there).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/tg_audio.h"
#include "readout_device.h"

using namespace tg;

namespace {
thread_local std::string g_audio_create_error;
constexpr int AU_MAX_K = 1024;
constexpr size_t AU_MAX_LDS = 96 * 1024;

struct AudioParams {
  int32_t E, Ls, T, K, KP, n_mat, slots;
  uint32_t key0, key1;
  double g_imp, g_scr;
  const int2* link_rng;     // [Ls] taxel range of each sensor link
  const double* coef;       // [n_mat + 1][slots][3] (a1, a2, g); bank n_mat is silent
  double* y1;               // [E * Ls][slots]
  double* y2;               // [E * Ls][slots]
  double* fn_prev;          // [E * Ls]
};

struct AudioLaunch {
  const float* ft;          // [S][6][E][T]
  const float* normal;      // [S][3][E][T]
  const int32_t* material;  // [E]
  float* out;               // [S][E][Ls][K]
  int64_t step0;
  int32_t n_steps;
};

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// the value of lane sub ^ 4 (rows of 16 lanes): row_shl:4 for the lower half of each group of 8,
// row_shr:4 for the upper half
__device__ __forceinline__ double xor4_d(double v, int sub) {
  const double up = dpp_d<0x104>(v), down = dpp_d<0x114>(v);
  return (sub & 4) ? down : up;
}
// sum over the G lanes of a pair (aligned groups of G lanes), the same in each of them
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if (G >= 2) v = v + dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
  if (G >= 4) v = v + dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
  if (G >= 8) v = v + dpp_d<0x141>(v);   // row_half_mirror: a lane of the other quad (all hold its sum)
  if (G >= 16) v = v + dpp_d<0x140>(v);  // row_mirror: a lane of the other group of 8
  return v;
}

// One sample of the pair's bank: advance this lane's resonators on u, return this lane's part of
// s[k] (the sum over its slots).
template <int MPL>
__device__ __forceinline__ double bank_part(double u, const double* a1, const double* a2n, const double* gg,
                                            double* y1, double* y2) {
  double part = 0.0;
#pragma unroll
  for (int i = 0; i < MPL; ++i) {
    const double y = fma(a1[i], y1[i], fma(a2n[i], y2[i], u));
    y2[i] = y1[i];
    y1[i] = y;
    part = fma(gg[i], y, part);
  }
  return part;
}
// Stage with bit `bit` of the partner: of the n values q[] (samples indexed by the bits not yet
// reduced), keep the half whose bit matches the lane's and add the partner's copy of it.
template <int N, int BIT>
__device__ __forceinline__ void transpose_stage(double* q, int sub) {
  const bool b = (sub & BIT) != 0;
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const double keep = b ? q[2 * i + 1] : q[2 * i], send = b ? q[2 * i] : q[2 * i + 1];
    double other;
    if constexpr (BIT == 1) other = dpp_d<0xB1>(send);        // quad_perm [1,0,3,2]
    else if constexpr (BIT == 2) other = dpp_d<0x4E>(send);   // quad_perm [2,3,0,1]
    else if constexpr (BIT == 4) other = xor4_d(send, sub);
    else other = dpp_d<0x128>(send);                          // row_ror:8 (lane sub ^ 8)
    q[i] = keep + other;
  }
}
// G samples' parts p[0..G) in each lane of a pair -> lane sub gets the pair's s[k0 + sub]: a
// transposed reduction, each exchange sending half of what the lane still holds.
template <int G>
__device__ __forceinline__ double group_transpose_sum(const double* p, int sub) {
  if constexpr (G == 1) {
    return p[0];
  } else {
    double q[G];
#pragma unroll
    for (int i = 0; i < G; ++i) q[i] = p[i];
    // after the stage of bit 2^j, q[i] holds sample (i << (j + 1)) | (sub & (2^(j+1) - 1)), summed
    // over the lanes that agree with sub above bit j
    transpose_stage<G, 1>(q, sub);
    if constexpr (G >= 4) transpose_stage<G / 2, 2>(q, sub);
    if constexpr (G >= 8) transpose_stage<G / 4, 4>(q, sub);
    if constexpr (G >= 16) transpose_stage<G / 8, 8>(q, sub);
    return q[0];
  }
}
}  // namespace

template <int G, int MPL>
__global__ __launch_bounds__(64) void tg_audio_kernel(const AudioParams p, const AudioLaunch q) {
  constexpr int PAIRS = 64 / G;
  extern __shared__ float rows[];   // [PAIRS][KP]
  __shared__ double red[G == 8 ? PAIRS * G * (G + 1) : 1];   // [pair][sample][lane] parts (rows padded)
  const int lane = threadIdx.x;
  const int pr = lane / G, sub = lane % G;
  const int64_t EL = (int64_t)p.E * p.Ls;
  const int64_t g0 = (int64_t)blockIdx.x * PAIRS;
  const int64_t g = g0 + pr;
  const bool live = g < EL;
  const int e = live ? (int)(g / p.Ls) : 0;
  const int l = live ? (int)(g - (int64_t)e * p.Ls) : 0;
  float* row = rows + pr * p.KP;

  int m = live ? q.material[e] : p.n_mat;
  if (m < 0 || m >= p.n_mat) m = p.n_mat;
  double a1[MPL], a2n[MPL], gg[MPL], y1[MPL], y2[MPL];
  const double* cf = p.coef + ((int64_t)m * p.slots + sub * MPL) * 3;
  const int64_t so = g * p.slots + sub * MPL;
#pragma unroll
  for (int i = 0; i < MPL; ++i) {
    a1[i] = cf[3 * i];
    a2n[i] = -cf[3 * i + 1];
    gg[i] = cf[3 * i + 2];
    y1[i] = live ? p.y1[so + i] : 0.0;
    y2[i] = live ? p.y2[so + i] : 0.0;
  }
  double fnp = live ? p.fn_prev[g] : 0.0;
  const int2 rng = p.link_rng[l];
  const int64_t ET = (int64_t)p.E * p.T;
  const int K = p.K, NC = (K + 3) >> 2;
  const int KG = K - K % G;   // samples in full groups of G

  for (int s = 0; s < q.n_steps; ++s) {
    // 1. excitation of the link
    double fn = 0.0, ftm = 0.0;
    if (live) {
      const float* f = q.ft + (int64_t)s * 6 * ET + (int64_t)e * p.T;
      const float* nm = q.normal + (int64_t)s * 3 * ET + (int64_t)e * p.T;
      for (int j = rng.x + sub; j < rng.y; j += G) {
        const double f0 = f[j], f1 = f[ET + j], f2 = f[2 * ET + j];
        const double m0 = nm[j], m1 = nm[ET + j], m2 = nm[2 * ET + j];
        const double dn = fma(f2, m2, fma(f1, m1, f0 * m0));
        const double t0 = fma(-dn, m0, f0), t1 = fma(-dn, m1, f1), t2 = fma(-dn, m2, f2);
        fn += dn;
        ftm += sqrt(fma(t2, t2, fma(t1, t1, t0 * t0)));
      }
    }
    fn = group_sum<G>(fn);
    ftm = group_sum<G>(ftm);
    const double d = fn - fnp;
    const double imp = p.g_imp * (d > 0.0 ? d : 0.0);
    fnp = fn;
    const double amp = p.g_scr * ftm;
    // 2. scrape noise into the row
    const uint32_t t = (uint32_t)(q.step0 + s);
    for (int c = sub; c < NC; c += G) {
      uint32_t x0 = (uint32_t)e, x1 = 0x80000000u + (uint32_t)l, x2 = t, x3 = (uint32_t)c;
      philox4x32_10(x0, x1, x2, x3, p.key0, p.key1);
      const uint32_t w[4] = {x0, x1, x2, x3};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 4 * c + i;
        if (k < K) row[k] = fmaf(2.f, u01(w[i]), -1.f);
      }
    }
    __syncthreads();
    // 3. the block's samples, G at a time (the next group's noise read ahead); the impact enters
    //    the first
    double extra = imp;
    float xn[G];
#pragma unroll
    for (int i = 0; i < G; ++i) xn[i] = KG > 0 ? row[i] : 0.f;
    for (int k0 = 0; k0 < KG; k0 += G) {
      float xc[G];
#pragma unroll
      for (int i = 0; i < G; ++i) xc[i] = xn[i];
      if (k0 + G < KG) {
#pragma unroll
        for (int i = 0; i < G; ++i) xn[i] = row[k0 + G + i];
      }
      double pk[G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        pk[i] = bank_part<MPL>(fma(amp, (double)xc[i], extra), a1, a2n, gg, y1, y2);
        extra = 0.0;
      }
      if constexpr (G == 8) {
        // the G parts of each sample through LDS: lane sub adds sample sub's parts in lane order
        // (one wave: its LDS writes land before its later reads).  At 8 lanes this beats the seven
        // DPP exchanges per 8 samples; at 16 the LDS bank conflicts make it slower, at 4 it ties.
        double* rd = red + pr * G * (G + 1);
#pragma unroll
        for (int i = 0; i < G; ++i) rd[i * (G + 1) + sub] = pk[i];
        double acc = rd[sub * (G + 1)];
#pragma unroll
        for (int ll = 1; ll < G; ++ll) acc += rd[sub * (G + 1) + ll];
        row[k0 + sub] = (float)acc;
      } else {
        row[k0 + sub] = (float)group_transpose_sum<G>(pk, sub);
      }
    }
    for (int k = KG; k < K; ++k) {
      const double v = group_sum<G>(bank_part<MPL>(fma(amp, (double)row[k], extra), a1, a2n, gg, y1, y2));
      extra = 0.0;
      if (sub == k - KG) row[k] = (float)v;
    }
    __syncthreads();
    // 4. the wave's rows to HBM
    float* o = q.out + ((int64_t)s * EL + g0) * K;
    const int nrow = (int)std::min<int64_t>(PAIRS, EL - g0);
    for (int r = 0; r < nrow; ++r)
      for (int k = lane; k < K; k += 64) __builtin_nontemporal_store(rows[r * p.KP + k], o + (int64_t)r * K + k);
    __syncthreads();
  }
  if (live) {
#pragma unroll
    for (int i = 0; i < MPL; ++i) {
      p.y1[so + i] = y1[i];
      p.y2[so + i] = y2[i];
    }
    if (sub == 0) p.fn_prev[g] = fnp;
  }
}

__global__ void tg_audio_zero_kernel(double* a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

struct tg_audio {
  AudioParams p{};
  int G = 1, mpl = 1;
  std::vector<void*> allocs;
  std::string err;
};

namespace {
tg_status afail(tg_audio* h, tg_status s, const std::string& msg) {
  if (h) h->err = msg; else g_audio_create_error = msg;
  return s;
}
template <class T>
hipError_t aalloc(tg_audio* h, T** p, size_t n) {
  void* q = nullptr;
  const hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
  if (e == hipSuccess) h->allocs.push_back(q);
  *p = (T*)q;
  return e;
}
bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
// the kernel instance of a lane layout (NULL for none)
const void* kernel_of(int G, int mpl) {
  switch (G * 16 + mpl) {
    case 17: return (const void*)tg_audio_kernel<1, 1>;
    case 18: return (const void*)tg_audio_kernel<1, 2>;
    case 20: return (const void*)tg_audio_kernel<1, 4>;
    case 24: return (const void*)tg_audio_kernel<1, 8>;
    case 33: return (const void*)tg_audio_kernel<2, 1>;
    case 34: return (const void*)tg_audio_kernel<2, 2>;
    case 36: return (const void*)tg_audio_kernel<2, 4>;
    case 40: return (const void*)tg_audio_kernel<2, 8>;
    case 65: return (const void*)tg_audio_kernel<4, 1>;
    case 66: return (const void*)tg_audio_kernel<4, 2>;
    case 68: return (const void*)tg_audio_kernel<4, 4>;
    case 72: return (const void*)tg_audio_kernel<4, 8>;
    case 129: return (const void*)tg_audio_kernel<8, 1>;
    case 130: return (const void*)tg_audio_kernel<8, 2>;
    case 132: return (const void*)tg_audio_kernel<8, 4>;
    case 257: return (const void*)tg_audio_kernel<16, 1>;
    case 258: return (const void*)tg_audio_kernel<16, 2>;
    default: return nullptr;
  }
}
hipError_t zero_state(const AudioParams& p, hipStream_t st) {
  const int64_t n[3] = {(int64_t)p.E * p.Ls * p.slots, (int64_t)p.E * p.Ls * p.slots, (int64_t)p.E * p.Ls};
  double* a[3] = {p.y1, p.y2, p.fn_prev};
  for (int i = 0; i < 3; ++i) {
    hipLaunchKernelGGL(tg_audio_zero_kernel, dim3((unsigned)((n[i] + 255) / 256)), dim3(256), 0, st, a[i], n[i]);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace

extern "C" {

tg_status tg_audio_create(const tg_audio_config* cfg, tg_audio** out) {
  if (!out) return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!cfg) return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "cfg is NULL");
  if (cfg->abi_version != TG_ABI_VERSION) return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "abi_version mismatch");
  const int E = cfg->num_envs, T = cfg->num_taxels, Ls = cfg->num_sensor_links, NM = cfg->num_materials;
  if (E < 1 || T < 1 || Ls < 1 || NM < 0) return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "sizes must be positive");
  if (!cfg->sensor_taxel_begin || !cfg->sensor_taxel_end || (NM > 0 && !cfg->materials))
    return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "NULL array");
  if ((int64_t)E * T * 6 >= (int64_t(1) << 31)) return afail(nullptr, TG_ERR_UNSUPPORTED, "E * T * 6 exceeds 2^31");
  if (cfg->slots < 1 || cfg->slots > 32) return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "slots must lie in 1..32");
  const int K = cfg->samples_per_step;
  if (K < 1 || K > AU_MAX_K) return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "samples_per_step must lie in 1..1024");
  if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt)) return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "dt must be > 0");
  if (!std::isfinite(cfg->g_imp) || !std::isfinite(cfg->g_scr))
    return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "non-finite gain");
  std::vector<int2> rng(Ls);
  for (int l = 0; l < Ls; ++l) {
    const int b = cfg->sensor_taxel_begin[l], en = cfg->sensor_taxel_end[l];
    if (b < 0 || en < b || en > T) return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "sensor link taxel range outside 0..T");
    rng[l] = make_int2(b, en);
  }
  // lanes per pair G and slots per lane MPL (powers of two, G * MPL >= slots): the smallest G
  // that gives every SIMD two waves, else the largest that fits.  The recurrence is a chain of
  // dependent FMAs per slot and the noise comes from LDS; with one wave per SIMD their latency
  // shows, and more lanes per pair cost more exchanges per sample (on the hand, 20480 pairs with
  // 16 slots, per 100-step launch: 3.7 ms at G = 2, 3.0 ms at G = 4, 2.9 ms at G = 8 with 2560
  // waves, 3.3 ms at G = 16).
  const int KP = ((K + 3) & ~3) + 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  const int64_t nsimd = 4 * (int64_t)cus, EL = (int64_t)E * Ls;
  int G = 0, mpl = 0;
  bool done = false;
  const int lp = cfg->lanes_per_pair;
  if (lp != 0 && lp != 1 && lp != 2 && lp != 4 && lp != 8 && lp != 16)
    return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "lanes_per_pair must be 0, 1, 2, 4, 8 or 16");
  for (int gl = 1; gl <= 16; gl *= 2) {
    if (cfg->lanes_per_pair != 0 && gl != cfg->lanes_per_pair) continue;
    int mp = 1;
    while (mp * gl < cfg->slots) mp *= 2;
    if (mp > 8 || (size_t)(64 / gl) * KP * sizeof(float) > AU_MAX_LDS) continue;
    const int64_t waves = (EL + 64 / gl - 1) / (64 / gl);
    if (G != 0 && done) continue;
    G = gl;
    mpl = mp;
    done = waves >= 2 * nsimd;
  }
  if (G == 0) return afail(nullptr, TG_ERR_UNSUPPORTED, "no lane layout fits the bank and the block in LDS");
  const int slots = G * mpl;
  const double dts = cfg->dt / (double)K;
  std::vector<double> coef((size_t)(NM + 1) * slots * 3, 0.0);
  for (int b = 0; b < NM; ++b) {
    const tg_audio_material& mt = cfg->materials[b];
    if (mt.num_modes < 0 || mt.num_modes > cfg->slots)
      return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "material " + std::to_string(b) + ": mode count outside 0..slots");
    if (mt.num_modes > 0 && (!mt.freq || !mt.decay || !mt.gain))
      return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "material " + std::to_string(b) + ": NULL array");
    for (int i = 0; i < mt.num_modes; ++i) {
      const double f = mt.freq[i], d = mt.decay[i], gn = mt.gain[i];
      if (!(f >= 0.0) || !std::isfinite(f) || !(d >= 0.0) || !std::isfinite(d) || !std::isfinite(gn))
        return afail(nullptr, TG_ERR_INVALID_ARGUMENT, "material " + std::to_string(b) + ": invalid mode");
      const double r = std::exp(-d * dts);
      double* c = &coef[((size_t)b * slots + i) * 3];
      c[0] = 2.0 * r * std::cos(2.0 * M_PI * f * dts);
      c[1] = r * r;
      c[2] = gn;
    }
  }
  tg_audio* h = new (std::nothrow) tg_audio();
  if (!h) return afail(nullptr, TG_ERR_OUT_OF_MEMORY, "host allocation failed");
  AudioParams& p = h->p;
  p.E = E; p.Ls = Ls; p.T = T; p.K = K; p.n_mat = NM; p.slots = slots;
  p.KP = KP;
  p.key0 = (uint32_t)cfg->seed;
  p.key1 = (uint32_t)(cfg->seed >> 32);
  p.g_imp = cfg->g_imp;
  p.g_scr = cfg->g_scr;
  h->G = G;
  h->mpl = mpl;
  int2* drng = nullptr;
  double *dcoef = nullptr, *y1 = nullptr, *y2 = nullptr, *fnp = nullptr;
  const size_t nst = (size_t)E * Ls * slots;
  hipError_t e = aalloc(h, &drng, Ls);
  if (e == hipSuccess) e = aalloc(h, &dcoef, coef.size());
  if (e == hipSuccess) e = aalloc(h, &y1, nst);
  if (e == hipSuccess) e = aalloc(h, &y2, nst);
  if (e == hipSuccess) e = aalloc(h, &fnp, (size_t)E * Ls);
  if (e == hipSuccess) e = hipMemcpy(drng, rng.data(), Ls * sizeof(int2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dcoef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice);
  p.link_rng = drng; p.coef = dcoef; p.y1 = y1; p.y2 = y2; p.fn_prev = fnp;
  if (e == hipSuccess && (size_t)(64 / G) * KP * sizeof(float) > 65536)
    e = hipFuncSetAttribute(kernel_of(G, mpl), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)((size_t)(64 / G) * KP * sizeof(float)));
  if (e == hipSuccess) e = zero_state(p, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    tg_audio_destroy(h);
    return afail(nullptr, TG_ERR_OUT_OF_MEMORY, std::string("device setup: ") + hipGetErrorString(e));
  }
  *out = h;
  return TG_OK;
}

tg_status tg_audio_rollout(tg_audio* h, const float* ft, const float* normal, const int32_t* material,
                           int64_t step0, int32_t n_steps, float* out, void* hip_stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->err.clear();
  if (!ft || !normal || !material || !out) return afail(h, TG_ERR_INVALID_ARGUMENT, "NULL buffer");
  if (n_steps < 0) return afail(h, TG_ERR_INVALID_ARGUMENT, "n_steps < 0");
  if (n_steps == 0) return TG_OK;
  if (step0 < 0 || step0 + n_steps > (int64_t(1) << 32))
    return afail(h, TG_ERR_INVALID_ARGUMENT, "steps must lie in [0, 2^32)");
  if (!aligned16(ft) || !aligned16(normal) || !aligned16(material) || !aligned16(out))
    return afail(h, TG_ERR_INVALID_ARGUMENT, "pointers must be 16-byte aligned");
  AudioLaunch q{};
  q.ft = ft; q.normal = normal; q.material = material; q.out = out;
  q.step0 = step0; q.n_steps = n_steps;
  const AudioParams& p = h->p;
  const int64_t EL = (int64_t)p.E * p.Ls;
  const int pairs = 64 / h->G;
  const dim3 grid((unsigned)((EL + pairs - 1) / pairs)), block(64);
  const size_t lds = (size_t)pairs * p.KP * sizeof(float);
  const hipStream_t st = (hipStream_t)hip_stream;
  const void* kf = kernel_of(h->G, h->mpl);
  if (!kf) return afail(h, TG_ERR_STATE, "lane layout");
  void* args[] = {(void*)&p, (void*)&q};
  const hipError_t el = hipLaunchKernel(kf, grid, block, args, lds, st);
  if (el != hipSuccess) return afail(h, TG_ERR_HIP, hipGetErrorString(el));
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? TG_OK : afail(h, TG_ERR_HIP, hipGetErrorString(e));
}

tg_status tg_audio_reset(tg_audio* h, void* hip_stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  h->err.clear();
  const hipError_t e = zero_state(h->p, (hipStream_t)hip_stream);
  return e == hipSuccess ? TG_OK : afail(h, TG_ERR_HIP, hipGetErrorString(e));
}

tg_status tg_audio_destroy(tg_audio* h) {
  if (!h) return TG_OK;
  for (void* p : h->allocs) (void)hipFree(p);
  delete h;
  return TG_OK;
}

const char* tg_audio_last_error(const tg_audio* h) { return h ? h->err.c_str() : g_audio_create_error.c_str(); }

}  // extern "C"
