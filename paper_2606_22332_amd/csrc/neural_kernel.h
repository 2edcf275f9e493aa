// Clean readout with the neural SDF surrogate (one object network per object) and the grid as
// the fallback inside a band around the surface.
//
// Per step, envs are first sorted by object id (tg_group_kernel), so that a workgroup that
// takes NEU_ENVS consecutive envs of that order keeps one object's packed BF16 network image in
// LDS and reloads it only when the object changes.  Inside an env, each wave takes groups of 64
// consecutive taxels:
//   probe        one taxel per lane: probe point, box test and x_hat;
//   tile phase   four MFMA tiles of 16 taxels, x_hat taken from the owning lanes by shuffles:
//                network forward (all four lane groups hold the 16 samples); where a taxel
//                needs a normal outside the band, the tile also runs the reverse pass for
//                d out / d x_hat;
//   readout phase one taxel per lane (lane group g keeps tile g's results): the grid lookup
//                where the point is far or |phi_nn| < band, then the same depth / normal /
//                force / proximity sequence as the grid path; contact bits by wave ballot; link
//                sums by segmented wave reductions into a per-wave slot in LDS, the four slots
//                added in wave order at the end of the env (bitwise repeatable).
#pragma once
#include "nsdf_device.h"
#include "readout_kernel.h"

namespace tg {

constexpr int NEU_THREADS = 256;
constexpr int NEU_ENVS = 8;

struct NBox {          // normalisation of an object's grid box
  float centre[3];
  float half, half_inv;
  float pad[3];
};

struct NLaunch {
  const KParams* kc;
  const NBox* boxes;
  const uint32_t* images;        // [n_obj][IMG_WORDS]
  const uint16_t* silu;          // SiLU table (global copy; staged in LDS)
  const int32_t* order;          // [E] envs sorted by object id (invalid ids last)
  float band;
  int64_t step;                  // unused by the clean readout; kept for symmetry
  const float* link_state;       // [13][E*L] of this step
  const float* obj_state;        // [13][E] or null
  const int32_t* obj_id;         // [E]
  unsigned long long* bits;      // [E][W]
  float* depth;                  // [E][T]
  float* prox;
  float* surfdist;
  float* ft;                     // [6][E][T]
  float* normal;                 // [3][E][T]
  float* link_sums;              // [11][L][E]
};

// Counting sort of the envs by object id (ids outside [0, n_obj) form the last bin); one
// workgroup of 1024 threads.  The order inside a bin is not significant.
__global__ __launch_bounds__(1024) void tg_group_kernel(const int32_t* __restrict__ obj_id, int E, int n_obj,
                                                         int32_t* __restrict__ order) {
  extern __shared__ int32_t cnt[];   // n_obj + 2
  const int nb = n_obj + 1;
  for (int i = threadIdx.x; i <= nb; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    const int o = obj_id[e];
    atomicAdd(&cnt[(o >= 0 && o < n_obj) ? o : n_obj], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < nb; ++i) {
      const int c = cnt[i];
      cnt[i] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    const int o = obj_id[e];
    const int pos = atomicAdd(&cnt[(o >= 0 && o < n_obj) ? o : n_obj], 1);
    order[pos] = e;
  }
}

__device__ __forceinline__ float wave_sum(float v) {
  v += __shfl_xor(v, 32);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 8);
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 1);
  return v;
}

__device__ __forceinline__ void pose_from_state(const float* st, int64_t col, int64_t stride, Pose& P) {
  P.p[0] = st[0 * stride + col]; P.p[1] = st[1 * stride + col]; P.p[2] = st[2 * stride + col];
  quat_to_R(st[3 * stride + col], st[4 * stride + col], st[5 * stride + col], st[6 * stride + col], P.R);
  P.v[0] = st[7 * stride + col]; P.v[1] = st[8 * stride + col]; P.v[2] = st[9 * stride + col];
  P.w[0] = st[10 * stride + col]; P.w[1] = st[11 * stride + col]; P.w[2] = st[12 * stride + col];
}

// Per-wave link-sum slots [wave][10][L]: they live in the unused middle of the static SiLU table
// (entries 2560..4095, 3 KB) when they fit there (L <= 19), else after the poses in dynamic LDS.
static_assert(NEU_THREADS == 256, "the link sums add four wave slots");
constexpr int NEU_HOLE_OFF = nsdf::SILU_NE * 128 * 2, NEU_HOLE_BYTES = nsdf::SILU_NEG * 2 - NEU_HOLE_OFF;
__host__ __device__ inline bool neural_sums_in_hole(int L) { return 4 * 10 * L * 4 <= NEU_HOLE_BYTES; }
// Dynamic LDS: image | link poses [L] | object pose | (link sums, when not in the table's hole);
// the SiLU table is a static array of SILU_BYTES beside it.
__host__ __device__ inline int neural_lds_bytes(int L) {
  return nsdf::IMG_BYTES + (L + 1) * (int)sizeof(Pose) + (neural_sums_in_hole(L) ? 0 : 4 * 10 * L * 4) + 16;
}

__global__ __launch_bounds__(NEU_THREADS, 2) void tg_neural_kernel(const NLaunch qarg) {
  using namespace nsdf;
  extern __shared__ __align__(16) uint8_t smem[];
  // launch arguments and handle constants through constant-address pointers refreshed per env:
  // scalar reloads instead of SGPRs pinned for the whole launch
  (void)qarg;
  typedef const __attribute__((address_space(4))) NLaunch* QPtr;
  typedef const __attribute__((address_space(4))) KParams* KcPtr;
  QPtr qp = (QPtr)__builtin_amdgcn_kernarg_segment_ptr();
  KcPtr kc = (KcPtr)qp->kc;
#define q (*qp)
#define p (*kc)
#define NEU_REFRESH() asm volatile("" : "+s"(kc), "+s"(qp))
  const int E = p.E, L = p.L, T = p.T, W = p.W;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, s = lane & 15;
  __shared__ __align__(16) uint16_t tab[SILU_ENTRIES];
  uint32_t* img = (uint32_t*)smem;
  for (int i = tid; i < SILU_ENTRIES / 2; i += NEU_THREADS) ((uint32_t*)tab)[i] = ((const uint32_t*)q.silu)[i];
  Pose* lpose = (Pose*)(smem + IMG_BYTES);
  Pose* opose = lpose + L;
  float* sums = neural_sums_in_hole(L) ? (float*)((uint8_t*)tab + NEU_HOLE_OFF) : (float*)(opose + 1);
  const Img im = img_at(smem);
  const int64_t EL = (int64_t)E * L, ET = (int64_t)E * T;
  int loaded = -1;
#pragma unroll 1
  for (int k = 0; k < NEU_ENVS; ++k) {
    NEU_REFRESH();
    const int idx = blockIdx.x * NEU_ENVS + k;
    if (idx >= E) break;                                   // uniform
    const int e = q.order[idx];
    const int oid = q.obj_id[e];
    const bool has = oid >= 0 && oid < p.n_obj;
    if (tid == 0) check_object_id(p.err, oid, p.n_obj);
    __syncthreads();                                       // LDS of the previous env is free
    if (has && oid != loaded) {
      const uint4* src = (const uint4*)(q.images + (size_t)oid * IMG_WORDS);
      for (int w = tid; w < IMG_BYTES / 16; w += NEU_THREADS) ((uint4*)img)[w] = src[w];
    }
    if (has) loaded = oid;
    for (int l = tid; l < L; l += NEU_THREADS) pose_from_state(q.link_state, (int64_t)e * L + l, EL, lpose[l]);
    if (q.obj_state && tid == NEU_THREADS - 1) pose_from_state(q.obj_state, e, E, *opose);
    for (int i = tid; i < (NEU_THREADS / 64) * 10 * L; i += NEU_THREADS) sums[i] = 0.f;
    __syncthreads();
    const Pose* Op = q.obj_state ? opose : nullptr;
    GridDesc gd;
    NBox bx;
    if (has) {
      gd = p.grids[oid];
      bx = q.boxes[oid];
    }
#pragma unroll 1
    for (int grp = wave; grp * 64 < T; grp += NEU_THREADS / 64) {
      const int j0 = grp * 64;
      // ---- probe of this lane's taxel j0 + lane (the tiles take theirs by lane shuffles) ----
      const int j = j0 + lane;
      const bool valid = j < T;
      const float4 ta = valid ? p.taxA[j] : make_float4(0.f, 0.f, 0.f, 0.f);
      const float4 tb = valid ? p.taxB[j] : make_float4(0.f, 0.f, 0.f, 0.f);
      const int l = valid ? __float_as_int(tb.w) : 0;
      const float xj[3] = {ta.x, ta.y, ta.z};
      float qw[3] = {0.f, 0.f, 0.f}, qo[3] = {0.f, 0.f, 0.f}, xh[3] = {0.f, 0.f, 0.f};
      bool far = false;
      float rnet = -INFINITY;   // R_j where the network may have to supply this taxel's normal
      if (has) {
        probe_point(lpose[l], Op, xj, qw, qo);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const float u = (qo[i] - gd.origin[i]) * gd.hinv;
          far |= !(u >= 0.f && u <= gd.nm1);
          xh[i] = (qo[i] - bx.centre[i]) * bx.half_inv;
        }
        if (valid && !far && ta.w > 0.f) rnet = ta.w;
      }
      // ---- tile phase: tile tt holds taxels j0 + 16 tt + (lane & 15) ----
      float my_phi = 0.f, my_g[3] = {0.f, 0.f, 0.f};
      if (has) {
#pragma unroll 1
        for (int tt = 0; tt < 4; ++tt) {
          const int src = 16 * tt + s;
          const float x0 = __shfl(xh[0], src), x1 = __shfl(xh[1], src), x2 = __shfl(xh[2], src);
          const float rj = __shfl(rnet, src);
          // a tile whose 16 taxels are all outside the box (or fillers) needs no network value
          if (!__any(rj > -INFINITY)) continue;
          uint32_t z[4][8];
          u32x4 pe[2];
          float a4[4][4];
          const float out = forward_tile(im, lane, x0, x1, x2, z, pe, a4, tab);
          const float phi_nn = bx.half * out;
          const bool need = !(fabsf(phi_nn) < q.band) && phi_nn < rj;
          float gx[3] = {0.f, 0.f, 0.f};
          if (__any(need)) input_grad_tile(im, lane, x0, x1, x2, z, gx);
          if (g == tt) {
            my_phi = phi_nn;
            my_g[0] = gx[0]; my_g[1] = gx[1]; my_g[2] = gx[2];
          }
        }
      }
      // ---- readout phase: lane <-> taxel j0 + lane ----
      TaxelOut o;
      taxel_out_clear(o);
      if (valid && has && ta.w > 0.f) {
        o.active = true;
        const Pose& Lp = lpose[l];
        if (far || fabsf(my_phi) < q.band) {
          GridHit h;
          grid_lookup(gd, p.grid_vals, qo, h);
          o.surf = h.surf;
          if (h.far) {
            o.far = true;
          } else {
            probe_finish(p, Lp, Op, xj, ta.w, tb, qw, h.phi,
                         [&](float& a, float& b, float& c) { grid_grad(h, a, b, c); }, o);
          }
        } else {
          o.surf = my_phi;
          probe_finish(p, Lp, Op, xj, ta.w, tb, qw, my_phi,
                       [&](float& a, float& b, float& c) { a = my_g[0]; b = my_g[1]; c = my_g[2]; }, o);
        }
      }
      const bool bit = o.depth > p.eta_on;
      const unsigned long long word = __ballot(bit);
      const int64_t et = (int64_t)e * T + j;
      if (valid) {
        if (q.depth) q.depth[et] = o.depth;
        if (q.prox) q.prox[et] = o.prox;
        if (q.surfdist) q.surfdist[et] = o.surf;
        if (q.ft) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            q.ft[c * ET + et] = o.f[c];
            q.ft[(3 + c) * ET + et] = o.tau[c];
          }
        }
        if (q.normal) {
#pragma unroll
          for (int c = 0; c < 3; ++c) q.normal[c * ET + et] = o.mb[c];
        }
      }
      if (q.bits && lane == 0) q.bits[(int64_t)e * W + (j0 >> 6)] = word;
      if (q.link_sums) {
        const float v[10] = {o.f[0], o.f[1], o.f[2], o.tau[0], o.tau[1], o.tau[2], bit ? 1.f : 0.f,
                             o.depth * tb.z, o.depth * tb.y, o.depth * tb.x};
        unsigned long long left = __ballot(valid);
#pragma unroll 1
        while (left) {                                     // one pass per link present in the wave
          const int lead = __ffsll((long long)left) - 1;
          const int lk = __shfl(l, lead);
          const bool sel = valid && l == lk;
#pragma unroll
          for (int c = 0; c < 10; ++c) {
            const float t = wave_sum(sel ? v[c] : 0.f);
            // this wave's own slot: its LDS adds complete in issue order, so the sum is fixed
            if (lane == 0) atomicAdd(&sums[(wave * 10 + c) * L + lk], t);
          }
          left &= ~__ballot(sel);
        }
      }
    }
    if (q.link_sums) {
      __syncthreads();
      for (int i = tid; i < 10 * L; i += NEU_THREADS) {
        const int c = i / L, l = i - c * L;
        const float a = ((sums[i] + sums[10 * L + i]) + sums[20 * L + i]) + sums[30 * L + i];
        const int64_t col = (int64_t)l * E + e;
        if (c < 6) {
          q.link_sums[c * EL + col] = a;
        } else if (c == 6) {
          q.link_sums[6 * EL + col] = a;
          q.link_sums[7 * EL + col] = a > 2.5f ? 1.f : 0.f;
        } else {
          q.link_sums[(c + 1) * EL + col] = 1.0e4f * a;
        }
      }
    }
  }
}

#undef q
#undef p
#undef NEU_REFRESH

}  // namespace tg
