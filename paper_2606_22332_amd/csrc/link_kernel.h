// The fused rollout kernel, organised by (link, env chunk) work items.
//
// A block owns one link l for `envs` consecutive environments and runs every step of the
// launch for them: lane r <-> (env el = r / np, taxel k = r % np), np = n_l rounded up to a
// multiple of 8, about 192..512 readouts per block whatever the link size, so uneven links waste
// few lanes, and two blocks share a CU so that one block's memory latency hides behind the
// other's arithmetic.  Because a block only ever sees one link, everything that couples taxels
// stays inside the block:
//   - dense crosstalk C_l Z_l runs on MFMA (16x16x32 BF16) with the six channels of all the
//     block's envs as the N columns; the link's A fragments are staged in LDS for the launch
//     (or read from L2 when they do not fit) and Z goes through an LDS staging area;
//   - banded crosstalk reads in-link neighbours from LDS;
//   - per-link sums (force/torque, contact count, agg_force) are reduced inside the block:
//     DPP sums over aligned 8-lane groups (each group inside one env), then one lane per
//     (channel, env) adds that env's group partials.
// The noise state (drift, lag / Maxwell, Schmitt bit, dead flag, stuck value, gain) of each
// readout lives in registers for the whole launch and touches HBM only at its ends.
//
// Per step (four barriers): the loader lanes build the rotation matrices from the pose scalars
// that were prefetched one per lane during the previous step; then the readout (probe point,
// gathers from the bricked grid, depth, contact, force/torque, proximity), its non-temporal
// stores (unit-stride runs of n_l floats per env), contact bits into LDS windows and the clean
// group sums; then the clean epilogue (bit words, link sums) and the crosstalk MFMA; then the
// noise chain and its outputs; then the noisy epilogue.
//
// The physical block id is remapped so that each of the 8 XCDs works through a contiguous
// range of items (neighbouring blocks share envs and their objects' bricks in that XCD's L2).
#pragma once
#include "readout_kernel.h"
#include "xtalk_dense.h"

namespace tg {

__device__ __forceinline__ void load_pose13(const float* base, int64_t stride, int64_t col, float* v) {
#pragma unroll
  for (int c = 0; c < 13; ++c) v[c] = base[c * stride + col];
}

__device__ __forceinline__ Pose pose_from13(const float* v) {
  Pose P;
  quat_to_R(v[3], v[4], v[5], v[6], P.R);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    P.p[i] = v[i];
    P.v[i] = v[7 + i];
    P.w[i] = v[10 + i];
  }
  return P;
}

// Outputs are written once and never read back by the kernel: non-temporal stores, so that the
// output stream does not evict the grid bricks the gathers reuse from L2.
// Non-temporal store through a uniform base (SGPR pair) and a per-lane 32-bit byte offset: the
// scalar-base form of the vector store, so no per-lane 64-bit address is formed.  (Outputs are
// never read by the kernel, so the store needs no ordering against its other memory accesses.)
__device__ __forceinline__ void store_at(float* base, uint32_t off4, float v) {
  asm volatile("global_store_dword %0, %1, %2 nt" : : "v"(off4), "v"(v), "s"(base));
}

// Two FP32 values rounded to BF16 (nearest even), packed low, high (one v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t bf16_pack2(float lo, float hi) {
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  typedef float f2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2){lo, hi}, bf2));
}

// Sum over each aligned group of 8 lanes (three DPP adds); the total is valid in the group's
// first lane, added as ((a0+a1)+(a2+a3))+((a4+a5)+(a6+a7)).  Called with every lane active.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float group8_sum(float v) {
  v = v + dpp_f<0xB1>(v);    // quad_perm [1,0,3,2]
  v = v + dpp_f<0x4E>(v);    // quad_perm [2,3,0,1]
  v = v + dpp_f<0x104>(v);   // row_shl:4 (lane i takes lane i + 4)
  return v;
}

// The 10 summed channels of one step (f, tau, contact, d * n_z, d * n_y, d * n_x), reduced over
// each 8-lane group and parked as P[ch][group] by the group's first lane, channel rows `stride`
// = groups + 1 floats apart: the reduction's lanes (channel, env) then read 10 different banks
// where a stride of 64 put every channel of an env on one bank.  An env's lanes are a whole
// number of groups (n_l padded to a multiple of 8), so every group belongs to one env; lanes
// outside a readout pass zeros.
__device__ __forceinline__ void put_group_sums(float* P, int stride, const float* v) {
  const bool lead = (threadIdx.x & 7) == 0;
  const int g = threadIdx.x >> 3;
  // the three DPP stages run across all ten channels in turn, so no stage reads a value written
  // by the instruction just before it (no hazard wait states between dependent DPP adds)
  float t[10];
#pragma unroll
  for (int c = 0; c < 10; ++c) t[c] = v[c] + dpp_f<0xB1>(v[c]);
#pragma unroll
  for (int c = 0; c < 10; ++c) t[c] = t[c] + dpp_f<0x4E>(t[c]);
#pragma unroll
  for (int c = 0; c < 10; ++c) t[c] = t[c] + dpp_f<0x104>(t[c]);
  if (lead) {
#pragma unroll
    for (int c = 0; c < 10; ++c) P[c * stride + g] = t[c];
  }
}

// A lane's roles in the per-step epilogues, fixed for the launch and packed in one register (byte
// fields): link sums (channel, env) for lane = channel * envs + env, bit words (env, word) for
// lane = env * nwin + word.  The plan gives every workgroup at least 14 lanes per env, so each
// epilogue takes a single pass and the integer divisions happen once, before the step loop.
__device__ __forceinline__ uint32_t lane_roles(int tid, int envs, int nwin) {
  const int rch = tid / envs, rel = tid - rch * envs;
  const int bel = tid / nwin, bw = tid - bel * nwin;
  const bool rok = rch < 10, bok = bel < envs;
  return (rok ? (uint32_t)rch | ((uint32_t)rel << 8) : 0xffffu) | (bok ? ((uint32_t)bel << 16) | ((uint32_t)bw << 24) : 0xffff0000u);
}

// Per-link observations of one step (App. B.2: summed force and torque, contact count, agg_bool,
// agg_force) from the group partials: one lane per (channel, env) item adds the env's groups in
// order; output [11][L][E], items env-fastest so neighbouring lanes store neighbouring floats.
template <class KP, class LI>
__device__ __forceinline__ void link_reduce(KP& p, LI& li, const float* P, int stride, int e0, int l,
                                            float* out, uint32_t roles) {
  const int gpe = li.np >> 3;
  const int64_t EL = (int64_t)p.E * p.L;
  {
    const int ch = roles & 0xffu, el = (roles >> 8) & 0xffu;
    if (ch >= 10) return;
    const int e = e0 + el;
    if (e >= p.E) return;
    const float* v = P + ch * stride + el * gpe;
    float acc = 0.f;
    for (int g = 0; g < gpe; ++g) acc += v[g];
    // byte offsets from the step's base: 11 * E * L * 4 fits 32 bits (checked at create)
    const uint32_t col = (uint32_t)l * (uint32_t)p.E + (uint32_t)e;
    const uint32_t el4 = (uint32_t)EL * 4u;
    const uint32_t o = (uint32_t)(ch < 7 ? ch : ch + 1) * el4 + col * 4u;
    store_at(out, o, ch < 7 ? acc : 1.0e4f * acc);
    if (ch == 6) store_at(out, o + el4, acc > 2.5f ? 1.f : 0.f);
  }
}

// Merge the LDS bit windows of this block's envs into the global [E][W] words of one step.  The
// words start at zero (cleared before the launch): a word inside this link is stored when it has
// a bit set; a word shared with a neighbouring link receives this link's nonzero bits by atomic or.
template <class KP, class LI>
__device__ __forceinline__ void store_bits(KP& p, LI& li, const unsigned* win, int e0,
                                           unsigned long long* out_step, uint32_t roles) {
  const int nw = li.nwin;
  const int wstart = li.off >> 6;
  const int lo = li.off, hi = li.off + li.n;
  {
    const int el = (roles >> 16) & 0xffu, w = roles >> 24;
    if (el >= li.envs) return;
    const int e = e0 + el;
    if (e >= p.E) return;
    const unsigned long long bits =
        (unsigned long long)win[(el * nw + w) * 2] | ((unsigned long long)win[(el * nw + w) * 2 + 1] << 32);
    const int gw = wstart + w;
    const int a = max(lo, gw * 64), b = min(hi, gw * 64 + 64);
    unsigned long long* dst = out_step + (int64_t)e * p.W + gw;
    if (a == gw * 64 && b == gw * 64 + 64) {
      if (bits) __builtin_nontemporal_store(bits, dst);
    } else {
      const int sh = a - gw * 64, len = b - a;
      const unsigned long long cov = (len >= 64 ? ~0ull : ((1ull << len) - 1ull)) << sh;
      const unsigned long long mine = bits & cov;
      if (mine) atomicOr(dst, mine);
    }
  }
}

// XT: crosstalk 0 none, 1 banded, 2 dense with the link's A fragments staged in LDS for the
// launch, 3 dense with them read from L2 each step (plans where they do not fit beside the rest).
// FULL = 0 compiles out the knobs none of the shipped workloads use (white noise, bias,
// quantisation, per-probe gain, probe-radius noise, normal / surface-distance outputs) so that
// the common path fits in 128 VGPRs (4 waves per SIMD) without spilling.
template <int NOISE, int XT, int HY, int OBJ, int FULL>
__global__ void __launch_bounds__(512, 4) tg_link_kernel(const KLaunch qarg) {
  // The handle's constants and this launch's arguments are read through constant-memory pointers
  // (the parameter block and the kernel-argument segment) that are made opaque at the top of
  // every step, so the compiler reloads them with scalar loads where they are used instead of
  // keeping all of them live in SGPRs across the whole step loop.
  (void)qarg;
  typedef const __attribute__((address_space(4))) KLaunch* QPtr;
  QPtr qp = (QPtr)__builtin_amdgcn_kernarg_segment_ptr();
  typedef const __attribute__((address_space(4))) KParams* KcPtr;   // constant memory: scalar loads
  KcPtr kc = (KcPtr)qp->kc;
#define q (*qp)
#define TG_REFRESH() asm volatile("" : "+s"(kc), "+s"(qp))
#define TG_REFRESH_PHASE() do {} while (0)
#define p (*kc)
  TG_REFRESH();
  extern __shared__ __align__(16) unsigned char smem[];
  // XCD-aware mapping of physical blocks to work items
  const int per = p.n_items_pad >> 3;
  const int item_id = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (item_id >= p.n_items) return;
  const int2 item = p.items[item_id];
  const int l = item.x, e0 = item.y;
  typedef const __attribute__((address_space(4))) LinkInfo* LiPtr;
  LiPtr lip = (LiPtr)(p.links + l);    // read where used; refreshed with the other pointers
#define li (*lip)
  const int n = li.n, envs = li.envs;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  LinkLds Ld;   // field by field: the source lives in the constant address space
  Ld.pose = p.lds.pose; Ld.opose = p.lds.opose; Ld.oid = p.lds.oid; Ld.bits = p.lds.bits; Ld.sums = p.lds.sums;
  Ld.xz = p.lds.xz; Ld.tax = p.lds.tax; Ld.gtab = p.lds.gtab; Ld.raw = p.lds.raw; Ld.bt = p.lds.bt; Ld.dt = p.lds.dt;
  Ld.afr = p.lds.afr; Ld.total = p.lds.total;
  Pose* lpose = (Pose*)(smem + Ld.pose);
  Pose* opose = (Pose*)(smem + Ld.opose);
  int* oids = (int*)(smem + Ld.oid);
  unsigned* bitw = (unsigned*)(smem + Ld.bits);
  float* S = (float*)(smem + Ld.sums);
  float* XZ = (float*)(smem + Ld.xz);
  float4* TX = (float4*)(smem + Ld.tax);     // [n][2]: (x_j, R_j), (n_j, link)
  GridDesc* GT = (GridDesc*)(smem + Ld.gtab);
  float* RAW = (float*)(smem + Ld.raw);      // [2][14][envs] prefetched step inputs
  const int winw = envs * li.nwin * 2;       // u32 words of one bit-window set

  const int np = li.np;                      // lanes per env (n padded to a multiple of 8)
  const int el = tid / np;
  const int k = tid - el * np;
  const int e = e0 + el;
  const bool act = el < envs && k < n && e < p.E;
  const int j = li.off + k;
  const int64_t ET = (int64_t)p.E * p.T;
  const int64_t EL = (int64_t)p.E * p.L;
  const int64_t kk = (int64_t)e * p.T + j;
  // byte offset of (e, j) in an [E][T] plane: fits 32 bits (checked at create), so every output
  // store is a uniform per-step base plus this fixed lane offset
  const uint32_t off4 = (uint32_t)kk * 4u;
  const uint32_t roles = lane_roles(tid, envs, li.nwin);

  for (int i = tid; i < n; i += nthr) {
    TX[2 * i] = p.taxA[li.off + i];
    TX[2 * i + 1] = p.taxB[li.off + i];
  }
  if (p.gtab_lds)
    for (int i = tid; i < p.n_obj; i += nthr) GT[i] = p.grids[i];
  // Step inputs: scalar c (13 link-pose values, then the object id) of env el at step s is
  // parked at RAW[(s&1)][c][el].  Lane i < 14*envs owns scalar (c = i / envs, el = i % envs)
  // for every step: one pointer and one per-step stride, fixed for the launch.
  // Offsets are packed in one int per lane: >= 0 into link_state (per step +13*E*L), < -1 the
  // object id -(off+2) (per step +E), -1 none.
  const int nraw = 14 * envs;
  int pf_off = -1;
  if (tid < nraw) {
    const int c = tid / envs, el_ = tid - c * envs;
    if (e0 + el_ < p.E) pf_off = c < 13 ? (int)(c * EL + (int64_t)(e0 + el_) * p.L + l) : -(e0 + el_) - 2;
  }
  auto prefetch = [&](int s_) -> float {
    if (pf_off >= 0) return q.link_state[(int64_t)s_ * 13 * EL + pf_off];
    return __int_as_float(q.obj_id[(int64_t)s_ * p.E + (-pf_off - 2)]);
  };
  if (pf_off != -1) RAW[tid] = prefetch(0);
  float D[6] = {0, 0, 0, 0, 0, 0}, Y[6] = {0, 0, 0, 0, 0, 0}, XP[6] = {0, 0, 0, 0, 0, 0};
  uint32_t yd2 = 0u, yd3 = 0u;               // carried-over pair of the drift stream
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
    if (FULL && p.has_gain) gain = p.gain[kk];
  }
  if (XT >= 2) {   // zero the B staging once: padding rows and columns stay zero
    uint32_t* bt = (uint32_t*)(smem + Ld.bt);
    for (int i = tid; i < (li.nt * 16 * li.kp) / 2; i += nthr) bt[i] = 0u;
    if (XT == 2) {   // the link's A fragments, read from LDS at every step
      uint4* af = (uint4*)(smem + Ld.afr);
      const uint4* src = p.xt_afrag + (int64_t)li.afrag_off * 64;
      for (int i = tid; i < li.mt * li.kt * 64; i += nthr) af[i] = src[i];
    }
  }
  const bool loader = tid < envs && e0 + tid < p.E;
  __syncthreads();   // LDS constants and the first step's inputs

  for (int s = 0; s < q.n_steps; ++s) {
    TG_REFRESH();
    asm volatile("" : "+s"(lip));
    const int64_t t = q.step0 + s;
    const int par = s & 1;
    Pose* lp = lpose + par * envs;
    Pose* op = opose + par * envs;
    int* oi = oids + par * envs;
    unsigned* bw = bitw + par * 2 * winw;
    unsigned* bwn = bw + winw;
    const float* rw = RAW + par * nraw;
    if (loader) {
      float pv[13];
#pragma unroll
      for (int c = 0; c < 13; ++c) pv[c] = rw[c * envs + tid];
      lp[tid] = pose_from13(pv);
      const int oid = __float_as_int(rw[13 * envs + tid]);
      oi[tid] = oid;
      check_object_id(p.err, oid, p.n_obj);
      if (OBJ) {
        load_pose13(q.obj_state + (int64_t)s * 13 * p.E, p.E, e0 + tid, pv);
        op[tid] = pose_from13(pv);
      }
    }
    for (int i = tid; i < 2 * winw; i += nthr) bw[i] = 0u;
    __syncthreads();   // B1: poses, ids, zeroed bit windows
    TG_REFRESH_PHASE();
    // prefetch this lane's scalar of the next step's inputs; parked in LDS before the last barrier
    const bool pre = s + 1 < q.n_steps;
    float rv = 0.f;
    if (pre && pf_off != -1) rv = prefetch(s + 1);

    const float4 ta = act ? TX[2 * k] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 tb = act ? TX[2 * k + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
    TaxelOut o;
    if (act) {
      readout_probe(p, GT, lp[el], OBJ ? &op[el] : nullptr, oi[el], ta, tb, o);
    } else {
      o.depth = 0.f; o.phi = 0.f; o.prox = 0.f; o.surf = 0.f; o.active = false; o.far = false;
#pragma unroll
      for (int i = 0; i < 3; ++i) { o.f[i] = 0.f; o.tau[i] = 0.f; o.mb[i] = 0.f; }
    }
    const bool bit = o.depth > p.eta_on;
    const int wbit = (li.off & 63) + k;   // bit position inside this env's window
    if (act) {
      if (q.depth) store_at(q.depth + (int64_t)s * ET, off4, o.depth);
      if (q.prox) store_at(q.prox + (int64_t)s * ET, off4, o.prox);
      if (FULL && q.surfdist) store_at(q.surfdist + (int64_t)s * ET, off4, o.surf);
      if (q.ft) {
        float* f = q.ft + (int64_t)s * 6 * ET;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          store_at(f + c * ET, off4, o.f[c]);
          store_at(f + (c + 3) * ET, off4, o.tau[c]);
        }
      }
      if (FULL && q.normal) {
        float* nm = q.normal + (int64_t)s * 3 * ET;
#pragma unroll
        for (int c = 0; c < 3; ++c) store_at(nm + c * ET, off4, o.mb[c]);
      }
      if (bit) atomicOr(&bw[el * li.nwin * 2 + (wbit >> 5)], 1u << (wbit & 31));
    }
    const bool sums = q.link_sums != nullptr;
    const int sstride = (nthr >> 3) + 1;   // channel stride of the group partials
    if (sums) {   // (o and tb are zero outside a readout)
      const float v[10] = {o.f[0], o.f[1], o.f[2], o.tau[0], o.tau[1], o.tau[2], bit ? 1.f : 0.f,
                           o.depth * tb.z, o.depth * tb.y, o.depth * tb.x};
      put_group_sums(S, sstride, v);
    }
    float z[6] = {gain * o.f[0], gain * o.f[1], gain * o.f[2], gain * o.tau[0], gain * o.tau[1], gain * o.tau[2]};
    if (NOISE && XT == 1) {
#pragma unroll
      for (int c = 0; c < 6; ++c) XZ[c * nthr + tid] = z[c];
    }
    if (NOISE && XT >= 2 && act) {
      const int kp = li.kp;
      uint16_t* brow = (uint16_t*)(smem + Ld.bt) + 6 * el * kp + k;   // column 6 el + c at c * kp
#pragma unroll
      for (int c = 0; c < 6; c += 2) {
        const uint32_t w = bf16_pack2(z[c], z[c + 1]);
        brow[c * kp] = (uint16_t)(w & 0xffffu);
        brow[(c + 1) * kp] = (uint16_t)(w >> 16);
      }
    }
    if (!NOISE && pre && pf_off != -1) RAW[(par ^ 1) * nraw + tid] = rv;   // the other parity is free
    __syncthreads();   // B2: clean bits, sums, crosstalk operands
    TG_REFRESH_PHASE();
    if (q.bits) store_bits(p, li, bw, e0, q.bits + (int64_t)s * p.E * p.W, roles);
    if (sums) link_reduce(p, li, S, sstride, e0, l, q.link_sums + (int64_t)s * 11 * EL, roles);

    if (NOISE) {
      if (XT >= 2) {
        // C_l Z on MFMA.  Wave w takes M tile w % MT and every G-th N tile (G = waves per M tile),
        // so it reads its A fragments (one per K tile; from LDS when the plan stages them, else
        // from L2) once per step.
        const uint16_t* bt = (const uint16_t*)(smem + Ld.bt);
        float* dt = (float*)(smem + Ld.dt);
        const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
        const int ncols = 6 * envs;
        const int G = nwaves >= li.mt ? nwaves / li.mt : 1;
        for (int mt = wave % li.mt; mt < li.mt && wave < G * li.mt; mt += nwaves) {
          const uint4* arow = p.xt_afrag + ((int64_t)li.afrag_off + (int64_t)mt * li.kt) * 64 + lane;
          const uint4* lrow = (const uint4*)(smem + Ld.afr) + mt * li.kt * 64 + lane;
          const uint4* asrc = XT == 2 ? lrow : arow;
          uint4 afr[4];   // K tiles 0..3 (links of up to 128 taxels) stay in registers
#pragma unroll
          for (int kt = 0; kt < 4; ++kt) afr[kt] = kt < li.kt ? asrc[kt * 64] : make_uint4(0u, 0u, 0u, 0u);
          // two N tiles per pass: independent accumulator chains interleave on the matrix core
          for (int nt = (nwaves >= li.mt ? wave / li.mt : 0); nt < li.nt; nt += 2 * G) {
            const int nt1 = nt + G;
            const bool two = nt1 < li.nt;
            const int col0 = nt * 16 + (lane & 15), col1 = nt1 * 16 + (lane & 15);
            const uint16_t* b0 = bt + col0 * li.kp + 8 * (lane >> 4);
            const uint16_t* b1 = bt + (two ? col1 : col0) * li.kp + 8 * (lane >> 4);
            f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
              if (kt < li.kt) {
                const bf16x8 a = __builtin_bit_cast(bf16x8, afr[kt]);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, *(const uint4*)(b0 + 32 * kt)),
                                                              acc0, 0, 0, 0);
                if (two)
                  acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, *(const uint4*)(b1 + 32 * kt)),
                                                                acc1, 0, 0, 0);
              }
            }
            for (int kt = 4; kt < li.kt; ++kt) {   // links of more than 128 taxels
              const bf16x8 a = __builtin_bit_cast(bf16x8, asrc[kt * 64]);
              acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, *(const uint4*)(b0 + 32 * kt)),
                                                            acc0, 0, 0, 0);
              if (two)
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, *(const uint4*)(b1 + 32 * kt)),
                                                              acc1, 0, 0, 0);
            }
            const int m0 = 16 * mt + 4 * (lane >> 4);
            if (col0 < ncols) {
#pragma unroll
              for (int r = 0; r < 4; ++r) dt[col0 * li.kpd + m0 + r] = acc0[r];
            }
            if (two && col1 < ncols) {
#pragma unroll
              for (int r = 0; r < 4; ++r) dt[col1 * li.kpd + m0 + r] = acc1[r];
            }
          }
        }
      }
      __syncthreads();   // B3: crosstalk results; the clean reduction is done with S
      TG_REFRESH_PHASE();
      float zt[6];
      if (XT == 1) {
        const float chi = p.chi;
        const bool hasl = k > 0, hasr = k < n - 1;
        const float cjj = 1.0f - chi * (float)((int)hasl + (int)hasr);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          float acc = cjj * z[c];
          if (act && hasl) acc = fmaf(chi, XZ[c * nthr + tid - 1], acc);
          if (act && hasr) acc = fmaf(chi, XZ[c * nthr + tid + 1], acc);
          zt[c] = acc;
        }
      } else if (XT >= 2) {
        const int kpd = li.kpd;
        const float* drow = (const float*)(smem + Ld.dt) + 6 * el * kpd + k;   // row 6 el + c at c * kpd
#pragma unroll
        for (int c = 0; c < 6; ++c) zt[c] = act ? drow[c * kpd] : 0.f;
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) zt[c] = z[c];
      }
      // Gaussian streams: one Philox call per step for channels 0-3, one per pair of steps for
      // channels 4-5 (its second pair is carried over to the odd step)
      const bool odd = (t & 1) != 0;
      float gd[6], gw[6];
      if (p.drift_sigma != 0.f) {
        gauss4(p.key0, p.key1, (uint32_t)e, (uint32_t)j, (uint32_t)t, 0u, gd);
        uint32_t ya, yb;
        if (!odd || s == 0) {
          uint32_t y0, y1, y2, y3;
          pair_call(p.key0, p.key1, (uint32_t)e, (uint32_t)j, (uint32_t)(t >> 1), 0u, y0, y1, y2, y3);
          ya = odd ? y2 : y0;
          yb = odd ? y3 : y1;
          yd2 = y2;
          yd3 = y3;
        } else {
          ya = yd2;
          yb = yd3;
        }
        box_muller(ya, yb, gd[4], gd[5]);
      }
      if (FULL && p.white_sigma != 0.f) {   // (both calls made every step)
        gauss4(p.key0, p.key1, (uint32_t)e, (uint32_t)j, (uint32_t)t, 2u, gw);
        uint32_t y0, y1, y2, y3;
        pair_call(p.key0, p.key1, (uint32_t)e, (uint32_t)j, (uint32_t)(t >> 1), 2u, y0, y1, y2, y3);
        box_muller(odd ? y2 : y0, odd ? y3 : y1, gw[4], gw[5]);
      }
      float fo[6];
      // The two lag rates as values in SGPRs: a per-lane choice between the two fields of the
      // constant block otherwise becomes a per-lane select of their addresses and six vector
      // loads per step.
      float k_load = 0.f, k_unload = 0.f;
      if (HY == 1) {
        k_load = p.kload;
        k_unload = p.kunload;
        asm volatile("" : "+s"(k_load), "+s"(k_unload));
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const float x = zt[c];
        float h = x;
        if (HY == 1) {
          const float kap = fabsf(x) > fabsf(Y[c]) ? k_load : k_unload;
          Y[c] = fmaf(kap, x - Y[c], Y[c]);
          h = Y[c];
        } else if (HY == 2) {
          Y[c] = fmaf(p.decay, Y[c], x - XP[c]);
          XP[c] = x;
          h = fmaf(p.beta, Y[c], x);
        }
        float v = h;
        if (FULL && p.bias != 0.f) v = v + p.bias;
        if (FULL && p.white_sigma != 0.f) v = fmaf(p.white_sigma, gw[c], v);
        if (p.drift_sigma != 0.f) {
          D[c] = fmaf(p.drift_sigma, gd[c], D[c]);
          v = v + D[c];
        }
        if (FULL && p.quant > 0.f) v = p.quant * rintf(v * p.qinv);
        if (dead) v = stuck;
        fo[c] = v;
      }
      if (act && q.ft_noisy) {
        float* f = q.ft_noisy + (int64_t)s * 6 * ET;
#pragma unroll
        for (int c = 0; c < 6; ++c) store_at(f + c * ET, off4, fo[c]);
      }
      float dd = o.depth;
      if (FULL && p.has_radius) {
        dd = 0.f;
        if (act && o.active && !o.far) {
          uint32_t x0 = (uint32_t)e, x1 = (uint32_t)j, x2 = (uint32_t)t, x3 = 6u;
          philox4x32_10(x0, x1, x2, x3, p.key0, p.key1);
          float Rn = ta.w + fmaf(u01(x0), p.two_rho, p.neg_rho);
          Rn = Rn > 0.f ? Rn : 0.f;
          const float df = Rn - o.phi;
          dd = df > 0.f ? df : 0.f;
        }
      }
      bool nb = (dd > p.eta_on) || (sch && dd > p.eta_off);
      if (dead) { nb = false; dd = 0.f; }
      sch = nb;
      if (act && nb) atomicOr(&bwn[el * li.nwin * 2 + (wbit >> 5)], 1u << (wbit & 31));
      const bool sums_n = q.link_sums_noisy != nullptr;
      if (sums_n) {
        const float4 tn = act ? TX[2 * k + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float v[10] = {act ? fo[0] : 0.f, act ? fo[1] : 0.f, act ? fo[2] : 0.f,
                             act ? fo[3] : 0.f, act ? fo[4] : 0.f, act ? fo[5] : 0.f,
                             act && nb ? 1.f : 0.f, dd * tn.z, dd * tn.y, dd * tn.x};
        put_group_sums(S, sstride, v);
      }
      if (pre && pf_off != -1) RAW[(par ^ 1) * nraw + tid] = rv;   // park the next step's inputs
      __syncthreads();   // B4: noisy bits and sums
      TG_REFRESH_PHASE();
      if (q.bits_noisy) store_bits(p, li, bwn, e0, q.bits_noisy + (int64_t)s * p.E * p.W, roles);
      if (sums_n) link_reduce(p, li, S, sstride, e0, l, q.link_sums_noisy + (int64_t)s * 11 * EL, roles);
    }
  }
  TG_REFRESH();
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

#undef p
#undef q
#undef li
#undef TG_REFRESH
#undef TG_REFRESH_PHASE
}  // namespace tg
