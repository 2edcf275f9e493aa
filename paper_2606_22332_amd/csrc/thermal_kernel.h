// Voxel temperature fields on the thermal links, integrated with the readout's rollout.
//
// One workgroup per field (env, thermal link), persistent over the launch's steps; each of its
// n*n = 256 threads owns one z-column of the 16^3 block and keeps it in registers for the whole
// rollout, so the field touches HBM only when the launch starts and ends.  Per step:
//   1. the link's taxels recompute their clean depth with the readout's own FP32 sequence (probe
//      point, grid lookup, d = [R_j - phi]_+), so the heat input uses exactly the depths the
//      readout reports;
//   2. each top-layer column sums kappa * d over the taxels above it, in taxel order;
//   3. columns exchange their values through LDS and apply the explicit step
//        s   = ((T[x-1] + T[x+1]) + (T[y-1] + T[y+1])) + (T[z-1] + T[z+1])   (mirrored faces)
//        src = (g + rho_f * faces * (T_amb - T)) [+ c_v * (T_obj - T) on the top layer]
//        T'  = T + (r * (s - 6 T) + src);
//   4. the temperature of the top-layer voxel under each taxel is written out.
#pragma once
#include "readout_kernel.h"

namespace tg {

constexpr int TH_N = 16;                 // voxels per axis handled by this kernel
constexpr int TH_THREADS = TH_N * TH_N;  // one thread per (x, y) column

struct ThermalParams {
  int32_t F;                   // fields per env
  const int32_t* field_link;   // [F]
  const int32_t* taxel_vox;    // [T] top-layer voxel (y * n + x) of thermal taxels, -1 otherwise
  const float* T_obj;          // [E]
  float* fields;               // [E][F][n^3], index ((z * n) + y) * n + x
  float r, g, rho_f, kappa, T_amb, T0;
  // the paper's step (App. D.1): spectral diffusion, T^4 radiation and convection, sensor lag
  int32_t spectral;
  const float* dct;            // [16][16] orthonormal DCT-II, row m: w_m cos(pi m (2i + 1) / 32)
  const float* hk;             // [3 * 15^2 + 1] h(s) = a k^2 / (1 + a k^2), k^2 = (pi / (n dx))^2 s
  float k_rad;                 // dt eps sigma / (rho c_p dx) per exposed face
  float k_conv;                // dt h / (rho c_p dx) per exposed face
  float lag;                   // dt / tau of the sensor element, 0 = no lag
  float* t_meas;               // [E][T] measured reading (state), when lag > 0
};

struct ThermalLaunch {
  const KParams* kc;
  const ThermalParams* th;
  int32_t n_steps;
  const float* link_state;     // [S][13][E*L]
  const float* obj_state;      // [S][13][E] or null
  const int32_t* obj_id;       // [S][E]
  float* temperature;          // [S][E][T] or null
  const float* depth;          // [S][E][T] the rollout's clean depths (written by the readout
                               // kernel before this launch), or null: recomputed here
};

// The paper's spectral diffusion step (App. D.1) on one 16^3 block.
// The mirror-padded FFT filter 1 / (1 + a k^2) is diagonal in the DCT-II basis C of the block, with
// k^2 = (pi / (n dx))^2 (mx^2 + my^2 + mz^2).  It is applied in the equal correction form
//   T' = T - C3^T (h * C3 (T - T0)),   h = a k^2 / (1 + a k^2) <= a k_max^2,
// so the rounding of the transforms multiplies only the small correction; T0 (the ambient
// temperature) changes nothing in exact arithmetic (C3 maps a constant to the mean mode alone, and
// h = 0 there) but keeps the transformed values small.  C3 is separable, and each axis is a 16 x 16
// matrix times a 16 x 256 matrix.  Each contraction runs on FP16 MFMA with both operands split into
// FP16 high and low parts (x = hi + lo, lo the FP16 rounding of x - hi, so hi + lo holds about 22
// bits): one v_mfma_f32_16x16x32_f16 takes [A_hi, A_hi] times [B_hi; B_lo] and a second takes
// [A_lo, A_lo] times the same B, so all four partial products accumulate in FP32, at a quarter of
// the matrix-core time of FP32 MFMA 16x16x4.  The block sits in the exchange buffer ex[z][y][x]
// (rows padded to 17 floats, planes 272): a contraction reads its B operand (the 16 values of the
// contracted axis for one column, 4 per lane group) straight from it and writes its 16 x 16 result
// back in place, each wave owning 4 whole tiles, so only the change of axis needs a barrier.  The
// forward x transform's result feeds the inverse x transform from registers: its 4 output rows per
// lane group are the inverse's K slice of that lane group.
//   lane l = 16 g + c:  A[i = c][k = 4 g + r],  B[k = 4 g + r][j = c],  D[i = 4 g + r][j = c]
// (register r; in the K = 32 operands slot r holds the high part of k = 4 g + r, slot 4 + r the
// low part of B, or a second copy of A's part).
typedef _Float16 dct_h8 __attribute__((ext_vector_type(8)));
typedef float dct_acc __attribute__((ext_vector_type(4)));
struct DctSplit {      // one lane's A operand of a 16 x 16 matrix: high and low FP16 parts
  dct_h8 hi, lo;
};
struct DctOperands {   // the DCT-II matrix C (forward) and C^T (inverse)
  DctSplit fwd;        // C[c][4 g + r]
  DctSplit inv;        // C^T[c][4 g + r] = C[4 g + r][c]
};
__device__ __forceinline__ DctSplit dct_split(const float v[4]) {
  DctSplit o;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const _Float16 h = (_Float16)v[r];
    const _Float16 lo = (_Float16)(v[r] - (float)h);
    o.hi[r] = h; o.hi[4 + r] = h;
    o.lo[r] = lo; o.lo[4 + r] = lo;
  }
  return o;
}
__device__ __forceinline__ DctOperands dct_operands(const float* dct, int lane) {
  const int g = lane >> 4, c = lane & 15;
  float f[4], v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    f[r] = dct[c * TH_N + 4 * g + r];
    v[r] = dct[(4 * g + r) * TH_N + c];
  }
  DctOperands o;
  o.fwd = dct_split(f);
  o.inv = dct_split(v);
  return o;
}
// D += A B for this lane's B values b[r] = B[4 g + r][c]
__device__ __forceinline__ dct_acc mfma_split(const DctSplit& A, const float b[4], dct_acc acc) {
  dct_h8 B;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const _Float16 h = (_Float16)b[r];
    B[r] = h;
    B[4 + r] = (_Float16)(b[r] - (float)h);
  }
  acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(A.hi, B, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(A.lo, B, acc, 0, 0, 0);
}
// One axis of a wave's 4 tiles: tile t reads B row k at ex[base(t) + k * ks + c * cs] and writes
// D row 4 g + r at ex[base(t) + (4 g + r) * ks + c * cs] (ks: stride of the contracted axis, cs:
// of the column axis).
__device__ __forceinline__ void dct_axis(float* ex, const DctSplit& A, int base0, int tstride, int ks, int cs,
                                         int lane) {
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int t = 0; t < 4; ++t) {   // (a tile's result goes back as soon as the MFMAs have read it)
    float* src = ex + base0 + t * tstride + c * cs;
    float b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) b[r] = src[(4 * g + r) * ks];
    const dct_acc z = {0.f, 0.f, 0.f, 0.f};
    const dct_acc d = mfma_split(A, b, z);
    src[(4 * g + 0) * ks] = d.x;
    src[(4 * g + 1) * ks] = d.y;
    src[(4 * g + 2) * ks] = d.z;
    src[(4 * g + 3) * ks] = d.w;
  }
}
// The step on a block held in the transforms' own layout: lane (g, c) of wave w keeps
// fv[4 t + r] = T(z = 4 g + r, y = 4 w + t, x = c), which is the forward z pass's B operand and
// the inverse z pass's D, so those two passes take their operand from registers and give their
// result back to them: two barriers and a third of the exchange-buffer traffic fewer per step.
__device__ __forceinline__ void spectral_diffuse_tiles(const DctOperands& C, const float* hk, float T0,
                                                       float fv[TH_N], float* ex, int tid) {
  constexpr int RS = TH_N + 1, PS = TH_N * (TH_N + 1);
  const int w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const dct_acc z0 = {0.f, 0.f, 0.f, 0.f};
  // forward z: tile t is the plane y = 4 w + t; K = z, columns x
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) b[r] = fv[4 * t + r] - T0;
    const dct_acc d = mfma_split(C.fwd, b, z0);
    float* dst = ex + (4 * w + t) * RS + c;
    dst[(4 * g + 0) * PS] = d.x;
    dst[(4 * g + 1) * PS] = d.y;
    dst[(4 * g + 2) * PS] = d.z;
    dst[(4 * g + 3) * PS] = d.w;
  }
  __syncthreads();
  // forward y: planes mz = 4 w + t; K = y (row stride), columns x
  dct_axis(ex, C.fwd, 4 * w * PS, PS, RS, 1, lane);
  __syncthreads();
  // forward x, scale by h, inverse x: planes mz = 4 w + t; K = x, columns my
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int mz = 4 * w + t;
    float* pl = ex + mz * PS;
    float b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) b[r] = pl[c * RS + 4 * g + r];
    const dct_acc acc = mfma_split(C.fwd, b, z0);
    const int b2 = c * c + mz * mz;
    float hb[4];
    hb[0] = acc.x * hk[(4 * g + 0) * (4 * g + 0) + b2];
    hb[1] = acc.y * hk[(4 * g + 1) * (4 * g + 1) + b2];
    hb[2] = acc.z * hk[(4 * g + 2) * (4 * g + 2) + b2];
    hb[3] = acc.w * hk[(4 * g + 3) * (4 * g + 3) + b2];
    const dct_acc inv = mfma_split(C.inv, hb, z0);
    pl[c * RS + 4 * g + 0] = inv.x;
    pl[c * RS + 4 * g + 1] = inv.y;
    pl[c * RS + 4 * g + 2] = inv.z;
    pl[c * RS + 4 * g + 3] = inv.w;
  }
  __syncthreads();
  // inverse y: planes mz = 4 w + t; K = my, columns x
  dct_axis(ex, C.inv, 4 * w * PS, PS, RS, 1, lane);
  __syncthreads();
  // inverse z into the registers: T' = T - correction
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float* src = ex + (4 * w + t) * RS + c;
    float b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) b[r] = src[(4 * g + r) * PS];
    const dct_acc d = mfma_split(C.inv, b, z0);
    fv[4 * t + 0] = fv[4 * t + 0] - d.x;
    fv[4 * t + 1] = fv[4 * t + 1] - d.y;
    fv[4 * t + 2] = fv[4 * t + 2] - d.z;
    fv[4 * t + 3] = fv[4 * t + 3] - d.w;
  }
  // (the exchange buffer is written again only after the step's later barrier)
}

// SPEC = 1: the paper's step (spectral diffusion, T^4 radiation and convection, sensor lag).  Both
// forms run at four waves per SIMD; the spectral one then spills some registers to scratch, which
// still beats two waves per SIMD without spills by a fifth.
template <int SPEC>
__global__ __launch_bounds__(TH_THREADS, 4) void tg_thermal_kernel(const ThermalLaunch q) {
  constexpr int n = TH_N;
  const KParams& p = *q.kc;
  const ThermalParams& th = *q.th;
  const int e = blockIdx.x / th.F, f = blockIdx.x - e * th.F;
  const int l = th.field_link[f];
  const int tid = threadIdx.x, x = tid % n, y = tid / n;
  const int E = p.E, L = p.L, T = p.T;
  const int64_t EL = (int64_t)E * L, ET = (int64_t)E * T;
  __shared__ float ex[n * n * (n + 1)];    // exchange buffer [z][y][x] (rows padded to 17 for the spectral step)
  __shared__ float cd[512];                // kappa * depth per taxel of the link
  __shared__ float top[n * n];
  __shared__ float cvs[SPEC ? n * n : 1];   // contact coefficient per top voxel (spectral step)
  __shared__ Pose lp, op;
  __shared__ int oid_s;
  // the spectral step's filter correction per |m|^2 and the DCT-II operands of this lane
  __shared__ float hks[SPEC ? 3 * (TH_N - 1) * (TH_N - 1) + 1 : 1];
  DctOperands dcto;
  if (SPEC) {
    dcto = dct_operands(th.dct, tid & 63);
    for (int i = threadIdx.x; i < 3 * (TH_N - 1) * (TH_N - 1) + 1; i += TH_THREADS) hks[i] = th.hk[i];
    __syncthreads();
  }
  float* fld = th.fields + ((int64_t)e * th.F + f) * (n * n * n);
  // the field in registers: a z-column per thread (x, y), or for the spectral step the transforms'
  // layout, col[4 t + r] = T(z = 4 g + r, y = 4 w + t, x = c) for lane (g, c) of wave w
  const int tw = tid >> 6, tg = (tid >> 4) & 3, tc = tid & 15;
  float col[n];
  if constexpr (SPEC) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) col[4 * t + r] = fld[((4 * tg + r) * n + 4 * tw + t) * n + tc];
  } else {
#pragma unroll
    for (int z = 0; z < n; ++z) col[z] = fld[(z * n + y) * n + x];
  }
  const int jb = __ldg(&p.link_off[l]), je = __ldg(&p.link_off[l + 1]);
  const int nl = je - jb;
  const float Tobj = th.T_obj[e];
  const float r = th.r, g = th.g, rf = th.rho_f, Tamb = th.T_amb;
  const int fxy = (x == 0) + (x == n - 1) + (y == 0) + (y == n - 1);
  const int myvox = y * n + x;
  // exchange-buffer slots of the four in-plane neighbours (at z = 0; + z n^2 for layer z); on a
  // face the voxel's own slot, which holds its current value: the mirrored neighbour, with no
  // per-voxel select
  const int sxm = x > 0 ? myvox - 1 : myvox, sxp = x < n - 1 ? myvox + 1 : myvox;
  const int sym = y > 0 ? myvox - n : myvox, syp = y < n - 1 ? myvox + n : myvox;
  // The taxels over this column's top voxel, in taxel order, found once for the launch: up to four
  // 16-bit indices packed in two registers (more than four: the per-step scan below).
  uint32_t mine01 = 0u, mine23 = 0u;
  int nmine = 0;
  for (int k = 0; k < nl; ++k)
    if (th.taxel_vox[jb + k] == myvox) {
      if (nmine < 2) mine01 |= (uint32_t)k << (16 * nmine);
      else if (nmine < 4) mine23 |= (uint32_t)k << (16 * (nmine - 2));
      ++nmine;
    }
  const int tvox = tid < nl ? th.taxel_vox[jb + tid] : 0;   // top voxel of taxel tid (one per lane)
  constexpr bool spec = SPEC != 0;
  // measured reading of taxel tid (the sensor element lag), kept in a register over the launch
  float tm = 0.f;
  if (spec && th.lag > 0.f && tid < nl) tm = th.t_meas[(int64_t)e * T + jb + tid];
  for (int s = 0; s < q.n_steps; ++s) {
    // 1. poses of this step (only to recompute the depths)
    if (!q.depth && tid == 0) {
      const float* ls = q.link_state + (int64_t)s * 13 * EL;
      const int64_t c = (int64_t)e * L + l;
      lp.p[0] = ls[0 * EL + c]; lp.p[1] = ls[1 * EL + c]; lp.p[2] = ls[2 * EL + c];
      quat_to_R(ls[3 * EL + c], ls[4 * EL + c], ls[5 * EL + c], ls[6 * EL + c], lp.R);
      oid_s = q.obj_id[(int64_t)s * E + e];
    }
    if (!q.depth && q.obj_state && tid == 1) {
      const float* os = q.obj_state + (int64_t)s * 13 * E;
      op.p[0] = os[0 * E + e]; op.p[1] = os[1 * E + e]; op.p[2] = os[2 * E + e];
      quat_to_R(os[3 * E + e], os[4 * E + e], os[5 * E + e], os[6 * E + e], op.R);
    }
    // 2. clean depth of the link's taxels: the readout's own output when the rollout writes it
    //    (each column reads its own taxels' depths below), else recomputed with the readout's
    //    FP32 sequence (the same value) into cd
    const float* dep = q.depth ? q.depth + (int64_t)s * ET + (int64_t)e * T + jb : nullptr;
    if (!dep) {
      __syncthreads();   // the poses of this step
      for (int k = tid; k < nl; k += TH_THREADS) {
        const int j = jb + k;
        const float4 ta = p.taxA[j];
        float d = 0.f;
        const int oid = oid_s;
        if (oid >= 0 && oid < p.n_obj && ta.w > 0.f) {
          const float xj[3] = {ta.x, ta.y, ta.z};
          float qw[3], qo[3];
          probe_point(lp, q.obj_state ? &op : nullptr, xj, qw, qo);
          GridHit h;
          grid_lookup(p.grids[oid], p.grid_vals, qo, h);
          if (!h.far) {
            const float diff = ta.w - h.phi;
            d = diff > 0.f ? diff : 0.f;
          }
        }
        cd[k] = th.kappa * d;
      }
      __syncthreads();
    }
    // 3. contact coefficient of this column's top voxel, in taxel order (kappa d per taxel, then
    //    the sum)
    auto coef = [&](int k) { return dep ? th.kappa * dep[k] : cd[k]; };
    float cv = 0.f;
    if (nmine <= 4) {
      if (nmine > 0) cv = cv + coef(mine01 & 0xffffu);
      if (nmine > 1) cv = cv + coef(mine01 >> 16);
      if (nmine > 2) cv = cv + coef(mine23 & 0xffffu);
      if (nmine > 3) cv = cv + coef(mine23 >> 16);
    } else {
      for (int k = 0; k < nl; ++k)
        if (th.taxel_vox[jb + k] == myvox) cv = cv + coef(k);
    }
    if constexpr (SPEC) {
      cvs[myvox] = cv;   // read by the lanes holding the top voxels, behind the transforms' barriers
      spectral_diffuse_tiles(dcto, hks, Tamb, col, ex, tid);
      // 4'. the paper's order after the diffusion: source, contact conduction on the top voxel,
      //     then radiation (T^4 in kelvin, as (T - Ta)(T_K + Ta_K)(T_K^2 + Ta_K^2)) and convection
      //     from every face of the block
      const float TaK = Tamb + 273.15f, TaK2 = TaK * TaK;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int yy = 4 * tw + t;
        const int fxy_t = (tc == 0) + (tc == n - 1) + (yy == 0) + (yy == n - 1);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int z = 4 * tg + rr;
          float tv = col[4 * t + rr] + g;
          if (z == n - 1) tv = tv + cvs[yy * n + tc] * (Tobj - tv);
          const int faces = fxy_t + (z == 0) + (z == n - 1);
          if (faces) {
            const float d = tv - Tamb, TK = tv + 273.15f;
            const float q4 = d * ((TK + TaK) * fmaf(TK, TK, TaK2));
            tv = tv - (float)faces * fmaf(th.k_rad, q4, th.k_conv * d);
          }
          col[4 * t + rr] = tv;
        }
        if (tg == 3) top[yy * n + tc] = col[4 * t + 3];
      }
    } else {
#pragma unroll
      for (int z = 0; z < n; ++z) ex[(z * n + y) * n + x] = col[z];
      __syncthreads();
      // 4. explicit step from the old values (exchange buffer, and registers for z +- 1): the
      //    column is updated in place from the bottom, with the old value below carried in `below`
      float below = col[0];
#pragma unroll
      for (int z = 0; z < n; ++z) {
        const float t = col[z];
        const float* ez = ex + z * n * n;
        const float xm = ez[sxm], xp = ez[sxp], ym = ez[sym], yp = ez[syp];
        const float zm = z > 0 ? below : t;
        const float zp = z < n - 1 ? col[z + 1] : t;
        const float sum = ((xm + xp) + (ym + yp)) + (zm + zp);
        const int faces = fxy + (z == 0) + (z == n - 1);
        const float rfx = rf * (float)faces;
        float src = g + rfx * (Tamb - t);
        if (z == n - 1) src = src + cv * (Tobj - t);
        below = t;
        col[z] = t + (r * (sum - 6.0f * t) + src);
      }
      top[myvox] = col[n - 1];
    }
    __syncthreads();   // every read of ex and cd is done; top is complete
    if (spec && th.lag > 0.f && tid < nl) tm = fmaf(th.lag, top[tvox] - tm, tm);
    if (q.temperature) {
      float* out = q.temperature + (int64_t)s * ET + (int64_t)e * T;
      if (tid < nl) out[jb + tid] = spec && th.lag > 0.f ? tm : top[tvox];
      for (int k = tid + TH_THREADS; k < nl; k += TH_THREADS) out[jb + k] = top[th.taxel_vox[jb + k]];
      if (f == 0)   // the first field's workgroup clears the taxels of the non-thermal links
        for (int j = tid; j < T; j += TH_THREADS)
          if (th.taxel_vox[j] < 0) out[j] = 0.f;
    }
  }
  if constexpr (SPEC) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) fld[((4 * tg + r) * n + 4 * tw + t) * n + tc] = col[4 * t + r];
  } else {
#pragma unroll
    for (int z = 0; z < n; ++z) fld[(z * n + y) * n + x] = col[z];
  }
  if (spec && th.lag > 0.f && tid < nl) th.t_meas[(int64_t)e * T + jb + tid] = tm;
}

__global__ void tg_thermal_reset_kernel(const ThermalParams* thp, int E, const uint8_t* mask) {
  const ThermalParams& th = *thp;
  const int64_t NV = (int64_t)TH_N * TH_N * TH_N;
  const int64_t total = (int64_t)E * th.F * NV;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int e = (int)(i / (th.F * NV));
  if (mask && !mask[e]) return;
  th.fields[i] = th.T0;
}

__global__ void tg_thermal_reset_meas_kernel(const ThermalParams* thp, int E, int T, const uint8_t* mask) {
  const ThermalParams& th = *thp;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)E * T) return;
  if (mask && !mask[i / T]) return;
  th.t_meas[i] = th.T0;
}

}  // namespace tg
