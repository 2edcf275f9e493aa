// Neural SDF surrogate: packing, training targets, gradient, Adam, fused training and
// evaluation kernels behind include/tg_nsdf.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tg_nsdf.h"
#include "nsdf_device.h"
#include "nsdf_host.h"

using namespace tg;
using namespace tg::nsdf;

namespace {
thread_local std::string g_nsdf_create_error;
constexpr int NT = 256;  // threads per workgroup: four waves

struct BoxDesc {      // per object: grid + normalisation of its box
  GridDesc grid;
  float centre[3];
  float half;         // e = (n-1) * spacing / 2
  float half_inv;     // RN(1 / e)
  float hi[3];        // far corner of the box
};
}  // namespace

// ------------------------------------------------------------------------------------------------
// packing: FP32 parameters -> per-object image (BF16 fragments + FP32 tail)
// ------------------------------------------------------------------------------------------------
__global__ void nsdf_pack_kernel(const float* __restrict__ P, int n_obj, uint32_t* __restrict__ img) {
  const int o = blockIdx.y;
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_obj || w >= IMG_WORDS) return;
  img[(size_t)o * IMG_WORDS + w] = image_word(P + (size_t)o * NPARAM, w);
}

// ------------------------------------------------------------------------------------------------
// training targets: clamp into the box, trilinear grid value, normalise
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ float grid_value(const GridDesc& gd, const float* __restrict__ vals, const float* q) {
  float t[3];
  int i[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float u = (q[d] - gd.origin[d]) * gd.hinv;
    const float uc = fminf(fmaxf(u, 0.0f), gd.nm1);
    const int ii = min((int)floorf(uc), gd.n - 2);
    i[d] = ii;
    t[d] = uc - (float)ii;
  }
  const int n = gd.n;
  const float* c = vals + gd.offset + ((int64_t)i[2] * n + i[1]) * n + i[0];
  const int sy = n, sz = n * n;
  const float c000 = c[0], c100 = c[1], c010 = c[sy], c110 = c[sy + 1];
  const float c001 = c[sz], c101 = c[sz + 1], c011 = c[sz + sy], c111 = c[sz + sy + 1];
  const float x00 = lerpf(t[0], c000, c100), x10 = lerpf(t[0], c010, c110);
  const float x01 = lerpf(t[0], c001, c101), x11 = lerpf(t[0], c011, c111);
  const float y0 = lerpf(t[1], x00, x10), y1 = lerpf(t[1], x01, x11);
  return lerpf(t[2], y0, y1);
}

// Analytic gradient of the same trilinear interpolant (App. A.1: the normal is the SDF gradient):
// the corner differences along each axis, interpolated over the other two, times 1/h.
__device__ __forceinline__ void grid_gradient(const GridDesc& gd, const float* __restrict__ vals, const float* q,
                                              float gr[3]) {
  float t[3];
  int i[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float u = (q[d] - gd.origin[d]) * gd.hinv;
    const float uc = fminf(fmaxf(u, 0.0f), gd.nm1);
    const int ii = min((int)floorf(uc), gd.n - 2);
    i[d] = ii;
    t[d] = uc - (float)ii;
  }
  const int n = gd.n;
  const float* c = vals + gd.offset + ((int64_t)i[2] * n + i[1]) * n + i[0];
  const int sy = n, sz = n * n;
  const float c000 = c[0], c100 = c[1], c010 = c[sy], c110 = c[sy + 1];
  const float c001 = c[sz], c101 = c[sz + 1], c011 = c[sz + sy], c111 = c[sz + sy + 1];
  const float x00 = lerpf(t[0], c000, c100), x10 = lerpf(t[0], c010, c110);
  const float x01 = lerpf(t[0], c001, c101), x11 = lerpf(t[0], c011, c111);
  const float y0 = lerpf(t[1], x00, x10), y1 = lerpf(t[1], x01, x11);
  const float dx0 = lerpf(t[1], c100 - c000, c110 - c010), dx1 = lerpf(t[1], c101 - c001, c111 - c011);
  gr[0] = lerpf(t[2], dx0, dx1) * gd.hinv;
  gr[1] = lerpf(t[2], x10 - x00, x11 - x01) * gd.hinv;
  gr[2] = (y1 - y0) * gd.hinv;
}

__global__ void nsdf_targets_kernel(const BoxDesc* __restrict__ boxes, const float* __restrict__ vals,
                                    const float* __restrict__ pts, int64_t n, float4* __restrict__ out,
                                    float4* __restrict__ gout) {
  const int o = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const BoxDesc b = boxes[o];
  const int64_t k = (int64_t)o * n + i;
  float q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) q[d] = fminf(fmaxf(pts[3 * k + d], b.grid.origin[d]), b.hi[d]);
  const float phi = grid_value(b.grid, vals, q);
  out[k] = make_float4((q[0] - b.centre[0]) * b.half_inv, (q[1] - b.centre[1]) * b.half_inv,
                       (q[2] - b.centre[2]) * b.half_inv, phi * b.half_inv);
  if (gout) {   // d phi / d q, which is also d(phi / e) / d x_hat
    float gr[3];
    grid_gradient(b.grid, vals, q, gr);
    gout[k] = make_float4(gr[0], gr[1], gr[2], 0.0f);
  }
}

// ------------------------------------------------------------------------------------------------
// loss gradient and training: one workgroup per object, four waves, wave w owns hidden layer w
// ------------------------------------------------------------------------------------------------
// A round takes 64 records, one tile of 16 per wave.  Each wave runs its tile forward and back
// through the network (input gradients on MFMA with the transposed fragments) and stages, for
// every layer, dz (BF16) and the layer's input activations (BF16) in LDS as [feature][sample].
// After a barrier, the owner of layer l contracts dz_l with the inputs of layer l over the 64
// samples (16x16x32 MFMA, K = samples of two tiles), so the weight gradient of each layer lives in
// one wave's accumulators for the whole step.  Bias gradients come from the same staged dz; the
// output layer's gradient is reduced through a small LDS buffer.
namespace {

constexpr int SROW = 20;                    // staging row: 16 samples + pad (u16), 40 bytes
constexpr int STAGE_U16 = 64 * SROW;        // one [64 feature][16 sample] buffer
constexpr int STAGE_BYTES = 4 * 4 * 2 * STAGE_U16 * 2;   // [wave][layer][dz | act]
constexpr int RED_FLOATS = 4 * 66 + 4;      // per wave: dw5[64], db5, loss; then the summed loss
static_assert(B5_OFF == W5_OFF + 64, "db5 follows dw5 in the parameter vector");
static_assert(STAGE_BYTES >= NPARAM * 4, "the step's gradient reuses the staging area");
// dynamic; with the static SiLU table (13,312 B) the kernel takes 161,328 B of the CU's 160 KiB
constexpr int LDS_FIT = IMG_BYTES + STAGE_BYTES + RED_FLOATS * 4;
static_assert(LDS_FIT + SILU_BYTES <= 160 * 1024, "fits one CU's LDS");

__device__ __forceinline__ uint16_t* stage_buf(uint8_t* smem, int wave, int l, int which) {
  return (uint16_t*)(smem + IMG_BYTES) + ((wave * 4 + l) * 2 + which) * STAGE_U16;
}

// Stage 16 values held in chain layout (B fragments b[2], lane group g, sample s) as rows of a
// [feature][sample] buffer.  pe = true: the encoding's own feature order (48 rows).
__device__ __forceinline__ void stage_frags(uint16_t* buf, const u32x4 b[2], int g, int s, bool pe) {
#pragma unroll
  for (int kt = 0; kt < 2; ++kt)
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const uint32_t w = b[kt][it >> 1];
      const uint16_t v = (uint16_t)((it & 1) ? (w >> 16) : (w & 0xffffu));
      int row;
      if (pe) {
        if (it >= 6) continue;
        row = 6 * (4 * kt + g) + it;
      } else {
        row = 32 * kt + chain_k(g, it);
      }
      buf[row * SROW + s] = v;
    }
}
// Eight samples of one feature row: four from each of two tiles (K order of a 16x16x32 MFMA).
__device__ __forceinline__ u32x4 stage_pair(const uint16_t* b0, const uint16_t* b1, int row, int g) {
  const u32x2 x = *(const u32x2*)(b0 + row * SROW + 4 * g);
  const u32x2 y = *(const u32x2*)(b1 + row * SROW + 4 * g);
  return u32x4{x[0], x[1], y[0], y[1]};
}

__device__ __forceinline__ float bf_sum8(u32x4 v) {
  return (bf_lo(v[0]) + bf_hi(v[0])) + (bf_lo(v[1]) + bf_hi(v[1])) + (bf_lo(v[2]) + bf_hi(v[2])) +
         (bf_lo(v[3]) + bf_hi(v[3]));
}

// Forward and backward of this wave's tile; stages dz and layer inputs of every layer.
// Samples 2i and 2i+1 of a tile (lanes s and s ^ 1) are a pair when pair_lambda > 0.
__device__ __forceinline__ void tile_backprop(const Img& im, uint8_t* smem, int wave, int lane, float4 rec, bool valid,
                                              float inv_n, float pair_lambda, float dw5[4][4], float& db5,
                                              float& loss, const uint16_t* tab) {
  const int g = lane >> 4, s = lane & 15;
  uint32_t z[4][8];
  u32x4 pe[2];
  float a4[4][4];
  const float out = forward_tile(im, lane, rec.x, rec.y, rec.z, z, pe, a4, tab);
  const float r = out - rec.w;
  float go = valid ? ((r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f)) * inv_n) : 0.f;
  float lp = fabsf(r);
  if (pair_lambda > 0.f) {   // uniform
    // d/d out of lambda |r_odd - r_even| is lambda sign(r_self - r_partner) on both members
    const float dr = r - __shfl_xor(r, 1);
    if (valid) go += pair_lambda * ((dr > 0.f ? 1.f : (dr < 0.f ? -1.f : 0.f)) * inv_n);
    if ((s & 1) == 0) lp += pair_lambda * fabsf(dr);
  }
  if (g == 0 && valid) {
    loss += lp;
    db5 += go;
  }
  float gr[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      dw5[m][q] = fmaf(go, a4[m][q], dw5[m][q]);
      gr[m][q] = go * im.tail[256 + 16 * m + 4 * g + q];
    }
#pragma unroll
  for (int l = 3; l >= 0; --l) {
    __builtin_amdgcn_sched_barrier(0);
    u32x4 db[2], ain[2];
    float dz[4][4];
    dz_frags(gr, z[l], db, dz);
    if (l == 0) {
      ain[0] = pe[0];
      ain[1] = pe[1];
    } else {
      act_frags_tab(z[l - 1], ain, tab);
    }
    stage_frags(stage_buf(smem, wave, l, 0), db, g, s, false);
    stage_frags(stage_buf(smem, wave, l, 1), ain, g, s, l == 0);
    if (l > 0) {
      f32x4 o[4];
      layer_bwd<4>(im, l, lane, db, o);
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) gr[m][q] = o[m][q];
    }
  }
}

// The same for a loss with the gradient term grad_lambda * sum_d |g_d - gt_d| (g = d out / d x_hat,
// gt the grid's gradient, grec.xyz).  With u = grad_lambda sign(g - gt) / n held fixed, the term's
// parameter gradient is that of u . g, the directional derivative of out along u, which a
// forward-mode tangent pass computes: adot_0 = J_enc u, zdot_l = W_l adot_l, adot_l+1 = silu'(z_l)
// zdot_l, u . g = w5 . adot_4.  Reverse mode through both chains gives per layer
//   zdbar = adbar silu'(z),  zbar = abar silu'(z) + adbar silu''(z) zdot,
//   dW_l += zbar a_l^T + zdbar adot_l^T,  db_l += zbar,  dw5 += go a_4 + adot_4,
// where adbar is the adjoint of the plain input-gradient pass (seed w5).  BF16 rounding as in the
// MFMA forward: the GEMM operands (adot_0..3, zdot, zbar, zdbar and the weights) are BF16, adot_4 and
// every sum FP32.  The LDS holds two staged operands per (wave, layer), so a round contracts twice:
// gs_first stages (zdbar, adot) and gs_second (zbar, a).  gs_second runs the input-gradient pass
// again beside the zbar chain (the same MFMA operands give the same adbar, bit for bit) instead of
// keeping its 48 FP32 values per lane alive across the first contraction.
__device__ __forceinline__ void gs_first(const Img& im, uint8_t* smem, int wave, int lane, float4 rec, float4 grec,
                                         bool valid, float inv_n, float pair_lambda, float grad_lambda,
                                         float dw5[4][4], float& db5, float& loss, const uint16_t* tab,
                                         uint32_t z[4][8], u32x4 pe[2], uint32_t zd[4][8], float& go) {
  const int g = lane >> 4, s = lane & 15;
  float a4[4][4];
  const float out = forward_tile(im, lane, rec.x, rec.y, rec.z, z, pe, a4, tab);
  const float r = out - rec.w;
  go = valid ? ((r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f)) * inv_n) : 0.f;
  float lp = fabsf(r);
  if (pair_lambda > 0.f) {   // uniform
    const float dr = r - __shfl_xor(r, 1);
    if (valid) go += pair_lambda * ((dr > 0.f ? 1.f : (dr < 0.f ? -1.f : 0.f)) * inv_n);
    if ((s & 1) == 0) lp += pair_lambda * fabsf(dr);
  }
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) dw5[m][q] = fmaf(go, a4[m][q], dw5[m][q]);
  // input-gradient pass (seed w5); its dz are zdbar, staged as the first operand
  float ad[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) ad[m][q] = im.tail[256 + 16 * m + 4 * g + q];
  f32x4 gf[3];
#pragma unroll
  for (int l = 3; l >= 0; --l) {
    __builtin_amdgcn_sched_barrier(0);
    u32x4 db[2];
    float dz[4][4];
    dz_frags(ad, z[l], db, dz);
    stage_frags(stage_buf(smem, wave, l, 0), db, g, s, false);
    if (l > 0) {
      f32x4 o[4];
      layer_bwd<4>(im, l, lane, db, o);
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) ad[m][q] = o[m][q];
    } else {
      layer_bwd<3>(im, 0, lane, db, gf);
    }
  }
  const float xs[3] = {rec.x, rec.y, rec.z};
  float gp[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) {   // feature f = 16m + 4g + q = 6k + 3c + d (c = 0 sine, 1 cosine)
      const int f = 16 * m + 4 * g + q;
      const int k = f / 6, rem = f - 6 * k, c = rem / 3, d = rem - 3 * c;
      const float t = __builtin_amdgcn_fractf((float)(1 << k) * 0.5f * xs[d]);
      const float w = (float)(1 << k) * 3.14159265358979323846f;
      const float dv = c == 0 ? w * __builtin_amdgcn_cosf(t) : -w * __builtin_amdgcn_sinf(t);
      const float contrib = gf[m][q] * dv;
      gp[0] += d == 0 ? contrib : 0.f;
      gp[1] += d == 1 ? contrib : 0.f;
      gp[2] += d == 2 ? contrib : 0.f;
    }
  const float gt[3] = {grec.x, grec.y, grec.z};
  float u[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float e = group_sum(gp[d]) - gt[d];
    lp += grad_lambda * fabsf(e);
    u[d] = valid ? grad_lambda * ((e > 0.f ? 1.f : (e < 0.f ? -1.f : 0.f)) * inv_n) : 0.f;
  }
  if (g == 0 && valid) {
    loss += lp;
    db5 += go;
  }
  // tangent pass along u: adot_l (BF16) staged as the second operand, zdot_l (BF16) kept
  u32x4 bin[2];
#pragma unroll
  for (int kt = 0; kt < 2; ++kt) {   // encoding order: lane group g of K-tile kt is frequency 4kt + g
    const int k = 4 * kt + g;
    const float sc = (float)(1 << k) * 0.5f, w = (float)(1 << k) * 3.14159265358979323846f;
    float v[6];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float t = __builtin_amdgcn_fractf(sc * xs[d]);
      v[d] = (w * __builtin_amdgcn_cosf(t)) * u[d];
      v[3 + d] = (-w * __builtin_amdgcn_sinf(t)) * u[d];
    }
    bin[kt] = u32x4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), 0u};
  }
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    __builtin_amdgcn_sched_barrier(0);
    stage_frags(stage_buf(smem, wave, l, 1), bin, g, s, l == 0);
    f32x4 acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) acc[m] = mfma32(frag(im.fwd, (l * 4 + m) * 2 + kt, lane), bin[kt], acc[m]);
    }
    float av[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      zd[l][2 * m] = pack2(acc[m][0], acc[m][1]);
      zd[l][2 * m + 1] = pack2(acc[m][2], acc[m][3]);
      const float zz[4] = {bf_lo(z[l][2 * m]), bf_hi(z[l][2 * m]), bf_lo(z[l][2 * m + 1]), bf_hi(z[l][2 * m + 1])};
      const float dd[4] = {bf_lo(zd[l][2 * m]), bf_hi(zd[l][2 * m]), bf_lo(zd[l][2 * m + 1]),
                           bf_hi(zd[l][2 * m + 1])};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float sg = sigmoid(zz[q]);
        av[m][q] = (sg * fmaf(zz[q], 1.0f - sg, 1.0f)) * dd[q];
      }
    }
    if (l < 3) {
#pragma unroll
      for (int kt = 0; kt < 2; ++kt)
        bin[kt] = u32x4{pack2(av[2 * kt][0], av[2 * kt][1]), pack2(av[2 * kt][2], av[2 * kt][3]),
                        pack2(av[2 * kt + 1][0], av[2 * kt + 1][1]), pack2(av[2 * kt + 1][2], av[2 * kt + 1][3])};
    } else {
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) dw5[m][q] = dw5[m][q] + av[m][q];
    }
  }
}

__device__ __forceinline__ void gs_second(const Img& im, uint8_t* smem, int wave, int lane, const uint32_t z[4][8],
                                          const u32x4 pe[2], const uint32_t zd[4][8], float go,
                                          const uint16_t* tab) {
  const int g = lane >> 4, s = lane & 15;
  float ab[4][4], ad[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ad[m][q] = im.tail[256 + 16 * m + 4 * g + q];
      ab[m][q] = go * ad[m][q];
    }
#pragma unroll
  for (int l = 3; l >= 0; --l) {
    __builtin_amdgcn_sched_barrier(0);
    // zbar (needs adbar) first; then zdbar, the next adbar and the next abar
    u32x4 db[2], dbd[2], ain[2];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
      uint32_t w[4], wd[4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = 2 * kt + h;
        const float zz[4] = {bf_lo(z[l][2 * m]), bf_hi(z[l][2 * m]), bf_lo(z[l][2 * m + 1]), bf_hi(z[l][2 * m + 1])};
        const float dd[4] = {bf_lo(zd[l][2 * m]), bf_hi(zd[l][2 * m]), bf_lo(zd[l][2 * m + 1]),
                             bf_hi(zd[l][2 * m + 1])};
        float zb[4], zdb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float sg = sigmoid(zz[q]);
          const float d1 = sg * fmaf(zz[q], 1.0f - sg, 1.0f);
          const float d2 = (sg * (1.0f - sg)) * fmaf(zz[q], 1.0f - 2.0f * sg, 2.0f);
          zdb[q] = ad[m][q] * d1;
          zb[q] = ab[m][q] * d1 + (ad[m][q] * d2) * dd[q];
        }
        w[2 * h] = pack2(zb[0], zb[1]);
        w[2 * h + 1] = pack2(zb[2], zb[3]);
        wd[2 * h] = pack2(zdb[0], zdb[1]);
        wd[2 * h + 1] = pack2(zdb[2], zdb[3]);
      }
      db[kt] = u32x4{w[0], w[1], w[2], w[3]};
      dbd[kt] = u32x4{wd[0], wd[1], wd[2], wd[3]};
    }
    stage_frags(stage_buf(smem, wave, l, 0), db, g, s, false);
    if (l == 0) {
      ain[0] = pe[0];
      ain[1] = pe[1];
    } else {
      act_frags_tab(z[l - 1], ain, tab);
    }
    stage_frags(stage_buf(smem, wave, l, 1), ain, g, s, l == 0);
    if (l > 0) {
      f32x4 o[4];
      layer_bwd<4>(im, l, lane, dbd, o);
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) ad[m][q] = o[m][q];
      layer_bwd<4>(im, l, lane, db, o);
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) ab[m][q] = o[m][q];
    }
  }
}

// Weight and bias gradient of layer L over the four staged tiles (owner wave only).
// bias = false: a second pass over other staged operands (the gradient term's zdbar against
// adot), which adds to the weight gradient only.
__device__ __forceinline__ void owner_wgrad(uint8_t* smem, int L, int lane, f32x4 acc[4][4], float dbp[4],
                                            bool bias) {
  const int g = lane >> 4, s = lane & 15;
  const int nin = L == 0 ? 3 : 4;
#pragma unroll
  for (int pr = 0; pr < 2; ++pr) {
    const uint16_t* d0 = stage_buf(smem, 2 * pr, L, 0);
    const uint16_t* d1 = stage_buf(smem, 2 * pr + 1, L, 0);
    const uint16_t* a0 = stage_buf(smem, 2 * pr, L, 1);
    const uint16_t* a1 = stage_buf(smem, 2 * pr + 1, L, 1);
    u32x4 A[4], B[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      A[m] = stage_pair(d0, d1, 16 * m + s, g);
      if (bias) dbp[m] += bf_sum8(A[m]);
    }
#pragma unroll
    for (int n = 0; n < 4; ++n)
      if (n < nin) B[n] = stage_pair(a0, a1, 16 * n + s, g);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n)
        if (n < nin) acc[m][n] = mfma32(A[m], B[n], acc[m][n]);
  }
}

__device__ __forceinline__ void adam_one(float& p, float& m, float& v, float g, float lr, float b1, float b2,
                                         float eps, float c1, float c2) {
  m = fmaf(b1, m, (1.0f - b1) * g);
  v = fmaf(b2, v, (1.0f - b2) * (g * g));
  p = p - lr * (m / c1) / (sqrtf(v / c2) + eps);
}

struct FitArgs {
  float* P;                 // [n_obj][NPARAM] FP32 parameters (updated when training)
  float* M;                 // Adam moments (training)
  float* V;
  const float4* samples;    // [n_obj][n] records
  int64_t n;
  float* grad;              // gradient output (gradient mode)
  float* loss;              // gradient mode: [n_obj]; training: [n_steps][n_obj] or null
  int64_t step0;
  int n_steps, n_obj, batch;
  float lr, b1, b2, eps;
  uint32_t key0, key1;
  float pair_lambda;        // > 0: records (2i, 2i+1) are pairs, loss adds lambda |r_odd - r_even|
  const float4* gsamples;   // [n_obj][n] grid gradients {d phi / d q, 0} (gradient term only)
  float grad_lambda;        // > 0: loss adds grad_lambda sum_d |g_d - gt_d| per record
  const uint16_t* silu;     // SiLU table (global copy; staged in LDS)
};

}  // namespace

template <int TRAIN, int GS>
__global__ __launch_bounds__(NT, 1) void nsdf_fit_kernel(const FitArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int o = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, s = lane & 15;
  const int L = wave;                                  // layer owned by this wave
  const int nin = L == 0 ? F : H;
  float* red = (float*)(smem + IMG_BYTES + STAGE_BYTES);
  float* Po = a.P + (size_t)o * NPARAM;
  const float4* So = a.samples + (size_t)o * a.n;
  const float4* Go = GS ? a.gsamples + (size_t)o * a.n : nullptr;
  for (int w = tid; w < IMG_WORDS; w += NT) ((uint32_t*)smem)[w] = image_word(Po, w);
  __shared__ __align__(16) uint16_t tab[SILU_ENTRIES];
  for (int i = tid; i < SILU_ENTRIES / 2; i += NT) ((uint32_t*)tab)[i] = ((const uint32_t*)a.silu)[i];
  const Img im = img_at(smem);
  const int64_t per_step = TRAIN ? a.batch : a.n;
  const float inv_n = 1.0f / (float)per_step;
  const int rounds = (int)((per_step + 63) / 64);
  const int n_steps = TRAIN ? a.n_steps : 1;
  for (int it = 0; it < n_steps; ++it) {
    const int64_t step = a.step0 + 1 + it;
    __syncthreads();
    f32x4 acc[4][4];
    float dbp[4], dw5[4][4], db5 = 0.f, lossp = 0.f;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      dbp[m] = 0.f;
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
        dw5[m][n] = 0.f;
      }
    }
    for (int rd = 0; rd < rounds; ++rd) {
      const int64_t j = (int64_t)rd * 64 + wave * 16 + s;
      bool valid;
      int64_t idx;
      if (TRAIN) {
        const bool pairs = a.pair_lambda > 0.f;   // uniform: draw pairs, lanes s and s ^ 1 share one
        const int64_t jj = pairs ? (j >> 1) : j;
        uint32_t x0 = (uint32_t)o, x1 = (uint32_t)step, x2 = (uint32_t)(jj >> 2), x3 = 8u;
        philox4x32_10(x0, x1, x2, x3, a.key0, a.key1);
        const uint32_t wsel = (jj & 3) == 0 ? x0 : ((jj & 3) == 1 ? x1 : ((jj & 3) == 2 ? x2 : x3));
        if (pairs) idx = 2 * (int64_t)(((uint64_t)wsel * (uint64_t)(a.n >> 1)) >> 32) + (j & 1);
        else idx = (int64_t)(((uint64_t)wsel * (uint64_t)a.n) >> 32);
        valid = true;
      } else {
        idx = j;
        valid = j < a.n;
      }
      const float4 rec = valid ? So[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
      if (GS) {
        const float4 grec = valid ? Go[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
        uint32_t z[4][8], zd[4][8];
        u32x4 pe[2];
        float go;
        gs_first(im, smem, wave, lane, rec, grec, valid, inv_n, a.pair_lambda, a.grad_lambda, dw5, db5, lossp, tab,
                 z, pe, zd, go);
        __syncthreads();
        owner_wgrad(smem, L, lane, acc, dbp, false);   // zdbar against adot
        __syncthreads();
        gs_second(im, smem, wave, lane, z, pe, zd, go, tab);
        __syncthreads();
        owner_wgrad(smem, L, lane, acc, dbp, true);    // zbar against a
      } else {
        tile_backprop(im, smem, wave, lane, rec, valid, inv_n, a.pair_lambda, dw5, db5, lossp, tab);
        __syncthreads();
        owner_wgrad(smem, L, lane, acc, dbp, true);
      }
      __syncthreads();
    }
    // Gradient of the step into LDS (the staging area is free now): owners write their layer,
    // the output layer is reduced over lanes and waves.
    float* Gl = (float*)(smem + IMG_BYTES);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        if (L == 0 && n == 3) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) Gl[W_OFF[L] + (16 * m + 4 * g + q) * nin + 16 * n + s] = acc[m][n][q];
      }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      float v = dbp[m];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (g == 0) Gl[B_OFF[L] + 16 * m + s] = v;
    }
    // Output layer and loss: each wave reduces its lanes and parks its partials (dw5, db5, loss)
    // in its own slot; the four slots are then added in wave order, so the step's gradient does
    // not depend on the order in which the waves arrive (training is bitwise repeatable).
    float* part = red + wave * 66;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float v = dw5[m][q];
        v += __shfl_xor(v, 8);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 1);
        if (s == 0) part[16 * m + 4 * g + q] = v;
      }
    {
      float v = db5, w = lossp;
#pragma unroll
      for (int k = 32; k >= 1; k >>= 1) {
        v += __shfl_xor(v, k);
        w += __shfl_xor(w, k);
      }
      if (lane == 0) {
        part[64] = v;
        part[65] = w;
      }
    }
    __syncthreads();
    if (tid < 66) {
      const float t = ((red[tid] + red[66 + tid]) + red[132 + tid]) + red[198 + tid];
      if (tid < 65) Gl[W5_OFF + tid] = t;   // dw5[0..63], then db5 at B5_OFF = W5_OFF + 64
      else red[264] = t;                    // loss
    }
    __syncthreads();
    if (!TRAIN) {
      float* G = a.grad + (size_t)o * NPARAM;
      for (int i = tid; i < NPARAM; i += NT) G[i] = Gl[i];
      if (a.loss && tid == 0) a.loss[o] = red[264] * inv_n;
    } else {
      float* Mo = a.M + (size_t)o * NPARAM;
      float* Vo = a.V + (size_t)o * NPARAM;
      const float c1 = (float)(1.0 - pow((double)a.b1, (double)step));
      const float c2 = (float)(1.0 - pow((double)a.b2, (double)step));
      float* tail = (float*)(smem + FWD_BYTES + BWD_BYTES);
#pragma unroll 1
      for (int i = tid; i < NPARAM; i += NT) {
        float p = Po[i], mm = Mo[i], vv = Vo[i];
        adam_one(p, mm, vv, Gl[i], a.lr, a.b1, a.b2, a.eps, c1, c2);
        Po[i] = p;
        Mo[i] = mm;
        Vo[i] = vv;
        int l = -1, oo = 0, in = 0;
        if (i < B_OFF[0]) { l = 0; oo = i / F; in = i - oo * F; }
        else if (i >= W_OFF[1] && i < B_OFF[1]) { l = 1; oo = (i - W_OFF[1]) >> 6; in = (i - W_OFF[1]) & 63; }
        else if (i >= W_OFF[2] && i < B_OFF[2]) { l = 2; oo = (i - W_OFF[2]) >> 6; in = (i - W_OFF[2]) & 63; }
        else if (i >= W_OFF[3] && i < B_OFF[3]) { l = 3; oo = (i - W_OFF[3]) >> 6; in = (i - W_OFF[3]) & 63; }
        if (l >= 0) {
          int fo, bo;
          weight_slots(l, oo, in, fo, bo);
          const uint16_t h16 = (uint16_t)bf16_bits(p);
          *(uint16_t*)(smem + fo) = h16;
          *(uint16_t*)(smem + bo) = h16;
        } else {
          int t;
          if (i == B5_OFF) t = 320;
          else if (i >= W5_OFF) t = 256 + (i - W5_OFF);
          else if (i >= B_OFF[3]) t = 192 + (i - B_OFF[3]);
          else if (i >= B_OFF[2]) t = 128 + (i - B_OFF[2]);
          else if (i >= B_OFF[1]) t = 64 + (i - B_OFF[1]);
          else t = i - B_OFF[0];
          tail[t] = p;
        }
      }
      if (a.loss && tid == 0) a.loss[(size_t)it * a.n_obj + o] = red[264] * inv_n;
    }
    __syncthreads();
  }
}

__global__ void nsdf_adam_kernel(float* __restrict__ P, float* __restrict__ M, float* __restrict__ V,
                                 const float* __restrict__ Gr, int64_t count, float lr, float b1, float b2, float eps,
                                 float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float p = P[i], m = M[i], v = V[i];
  adam_one(p, m, v, Gr[i], lr, b1, b2, eps, c1, c2);
  P[i] = p;
  M[i] = m;
  V[i] = v;
}

// Evaluation: one workgroup per (object, chunk of 64*k points), image of that object in LDS.
constexpr int QUERY_TILES_PER_WAVE = 8;
// trace (or null): per point [5][64] BF16 bits, row 0 the 48 encoding features (feature order of
// the encoding), rows 1..4 the BF16 pre-activations of the four hidden layers (unit order).
__global__ __launch_bounds__(NT) void nsdf_query_kernel(const uint32_t* __restrict__ images,
                                                        const int64_t* __restrict__ offsets,
                                                        const float* __restrict__ xhat, float* __restrict__ out,
                                                        float* __restrict__ grad, const uint16_t* __restrict__ silu,
                                                        uint16_t* __restrict__ trace) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int o = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t beg = offsets[o], end = offsets[o + 1];
  const int64_t chunk = (int64_t)blockIdx.x * (4 * 16 * QUERY_TILES_PER_WAVE);
  if (beg + chunk >= end) return;  // uniform over the workgroup
  uint32_t* img = (uint32_t*)smem;
  const uint32_t* src = images + (size_t)o * IMG_WORDS;
  for (int w = tid; w < IMG_WORDS; w += NT) img[w] = src[w];
  __shared__ __align__(16) uint16_t tab[SILU_ENTRIES];
  for (int i = tid; i < SILU_ENTRIES / 2; i += NT) ((uint32_t*)tab)[i] = ((const uint32_t*)silu)[i];
  __syncthreads();
  const Img im = img_at(smem);
  for (int tt = 0; tt < QUERY_TILES_PER_WAVE; ++tt) {
    const int64_t i = beg + chunk + ((int64_t)(wave * QUERY_TILES_PER_WAVE + tt) * 16) + (lane & 15);
    if (beg + chunk + (int64_t)(wave * QUERY_TILES_PER_WAVE + tt) * 16 >= end) break;  // wave-uniform
    const bool valid = i < end;
    float x0 = 0.f, x1 = 0.f, x2 = 0.f;
    if (valid) {
      x0 = xhat[3 * i];
      x1 = xhat[3 * i + 1];
      x2 = xhat[3 * i + 2];
    }
    uint32_t z[4][8];
    u32x4 pe[2];
    float a4[4][4];
    const float y = forward_tile(im, lane, x0, x1, x2, z, pe, a4, tab);
    float gx[3] = {0.f, 0.f, 0.f};
    if (grad) input_grad_tile(im, lane, x0, x1, x2, z, gx);
    if (trace && valid) {
      const int g = lane >> 4;
      uint16_t* tr = trace + i * 320;
#pragma unroll
      for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int it = 0; it < 6; ++it) {
          const uint32_t w = pe[kt][it >> 1];
          tr[6 * (4 * kt + g) + it] = (uint16_t)((it & 1) ? (w >> 16) : (w & 0xffffu));
        }
#pragma unroll
      for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint32_t w = z[l][2 * m + (r >> 1)];
            tr[64 * (l + 1) + 16 * m + 4 * g + r] = (uint16_t)((r & 1) ? (w >> 16) : (w & 0xffffu));
          }
    }
    if (valid && lane < 16) {
      out[i] = y;
      if (grad) {
        grad[3 * i] = gx[0];
        grad[3 * i + 1] = gx[1];
        grad[3 * i + 2] = gx[2];
      }
    }
  }
}

// ------------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------------
struct tg_nsdf {
  int n_obj = 0;
  int device = -1;              // current device at create: every buffer below lives there
  BoxDesc* d_boxes = nullptr;
  float* d_vals = nullptr;
  uint32_t* d_img = nullptr;
  uint16_t* d_silu = nullptr;
  std::string err;
};

namespace {
tg_status nfail(tg_nsdf* h, tg_status s, const std::string& msg) {
  if (h) h->err = msg; else g_nsdf_create_error = msg;
  return s;
}
bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
}  // namespace

hipError_t nsdf_pack_images(const float* params, int n_obj, uint32_t* images, hipStream_t stream) {
  hipLaunchKernelGGL(nsdf_pack_kernel, dim3((IMG_WORDS + 255) / 256, n_obj), dim3(256), 0, stream, params, n_obj,
                     images);
  return hipGetLastError();
}

// Pack the parameters into per-object images at img, then evaluate the points (both launches on
// the caller's stream).  Shared by the handle's own image buffer and the static one below.
static tg_status launch_query(tg_nsdf* h, uint32_t* img, const float* params, const int64_t* offsets,
                              int64_t max_count, const float* xhat, float* out, float* grad, hipStream_t s,
                              uint16_t* trace = nullptr) {
  hipLaunchKernelGGL(nsdf_pack_kernel, dim3((IMG_WORDS + 255) / 256, h->n_obj), dim3(256), 0, s, params, h->n_obj,
                     img);
  if (max_count > 0) {
    const int64_t per_block = 4 * 16 * QUERY_TILES_PER_WAVE;
    const dim3 grid((unsigned)((max_count + per_block - 1) / per_block), (unsigned)h->n_obj);
    hipLaunchKernelGGL(nsdf_query_kernel, grid, dim3(NT), IMG_BYTES, s, img, offsets, xhat, out, grad, h->d_silu,
                       trace);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? TG_OK : nfail(h, TG_ERR_HIP, hipGetErrorString(e));
}

// Images for the allocation-free evaluation: one static device array per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the host that name is
// only a stand-in for the symbol); it uses the device address that hipGetSymbolAddress returns,
// looked up once per device and kept in g_scratch_addr.
static __device__ __align__(256) uint32_t scratch[(size_t)TG_NSDF_QUERY_NOALLOC_MAX_OBJECTS * IMG_WORDS];
static_assert((size_t)TG_NSDF_QUERY_NOALLOC_MAX_OBJECTS * IMG_BYTES == TG_NSDF_QUERY_NOALLOC_SCRATCH_BYTES,
              "header states the static scratch size");

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_addr[MAX_DEVICES] = {};

// Device address of this GPU's scratch array (the current device), looked up on first use.
tg_status scratch_addr(tg_nsdf* h, int dev, uint32_t** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return nfail(h, TG_ERR_UNSUPPORTED, "query_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return nfail(h, TG_ERR_HIP, std::string("query_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch_addr[dev] = (uint32_t*)p;
  }
  *out = g_scratch_addr[dev];
  return TG_OK;
}
}  // namespace

namespace {
// Checks shared by the gradient and training entry points; nullptr when the arguments are valid.
const char* loss_terms_error(int64_t n, float pair_lambda, float grad_lambda, const float* samples,
                             const float* grad_samples) {
  if (!(pair_lambda >= 0.f) || (pair_lambda > 0.f && (n & 1)))
    return "pair_lambda must be >= 0, with an even n when > 0";
  if (!(grad_lambda >= 0.f) || (grad_lambda > 0.f && !grad_samples))
    return "grad_lambda must be >= 0, with grad_samples when > 0";
  if (!aligned16(samples) || (grad_lambda > 0.f && !aligned16(grad_samples))) return "samples not 16-byte aligned";
  return nullptr;
}

template <int TRAIN, int GS>
tg_status launch_fit(tg_nsdf* h, const FitArgs& a, hipStream_t stream) {
  hipError_t e = hipFuncSetAttribute((const void*)nsdf_fit_kernel<TRAIN, GS>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, LDS_FIT);
  if (e != hipSuccess) return nfail(h, TG_ERR_HIP, hipGetErrorString(e));
  hipLaunchKernelGGL((nsdf_fit_kernel<TRAIN, GS>), dim3(h->n_obj), dim3(NT), LDS_FIT, stream, a);
  e = hipGetLastError();
  return e == hipSuccess ? TG_OK : nfail(h, TG_ERR_HIP, hipGetErrorString(e));
}
}  // namespace

extern "C" {

tg_status tg_nsdf_create(const tg_nsdf_config* cfg, tg_nsdf** out) {
  if (!out) return nfail(nullptr, TG_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!cfg) return nfail(nullptr, TG_ERR_INVALID_ARGUMENT, "cfg is NULL");
  if (cfg->abi_version != TG_ABI_VERSION) return nfail(nullptr, TG_ERR_INVALID_ARGUMENT, "abi_version mismatch");
  if (cfg->num_objects < 1 || !cfg->grids) return nfail(nullptr, TG_ERR_INVALID_ARGUMENT, "no objects");
  std::vector<BoxDesc> boxes(cfg->num_objects);
  int64_t total = 0;
  for (int o = 0; o < cfg->num_objects; ++o) {
    const tg_sdf_grid& g = cfg->grids[o];
    if (g.n < 2 || !(g.spacing > 0.f) || !g.values)
      return nfail(nullptr, TG_ERR_INVALID_ARGUMENT, "grid " + std::to_string(o) + " invalid");
    BoxDesc& b = boxes[o];
    for (int d = 0; d < 3; ++d) b.grid.origin[d] = g.origin[d];
    b.grid.spacing = g.spacing;
    b.grid.hinv = 1.0f / g.spacing;
    b.grid.nm1 = (float)(g.n - 1);
    b.grid.n = g.n;
    b.grid.nb = 0;        // plain x-fastest order here (grid_value), not bricks
    b.grid.offset = total;
    const float ext = (float)(g.n - 1) * g.spacing;
    b.half = 0.5f * ext;
    b.half_inv = 1.0f / b.half;
    for (int d = 0; d < 3; ++d) {
      b.centre[d] = g.origin[d] + b.half;
      b.hi[d] = g.origin[d] + ext;
    }
    total += (int64_t)g.n * g.n * g.n;
  }
  tg_nsdf* h = new (std::nothrow) tg_nsdf();
  if (!h) return nfail(nullptr, TG_ERR_OUT_OF_MEMORY, "host allocation failed");
  h->n_obj = cfg->num_objects;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return nfail(nullptr, TG_ERR_HIP, "hipGetDevice failed");
  }
  if (hipMalloc(&h->d_boxes, sizeof(BoxDesc) * boxes.size()) != hipSuccess ||
      hipMalloc(&h->d_vals, sizeof(float) * total) != hipSuccess ||
      hipMalloc(&h->d_img, (size_t)IMG_BYTES * h->n_obj) != hipSuccess ||
      hipMalloc(&h->d_silu, SILU_BYTES) != hipSuccess) {
    tg_nsdf_destroy(h);
    return nfail(nullptr, TG_ERR_OUT_OF_MEMORY, "device allocation failed");
  }
  std::vector<uint16_t> silu(SILU_ENTRIES);
  build_silu_table(silu.data());
  hipError_t e = hipMemcpy(h->d_boxes, boxes.data(), sizeof(BoxDesc) * boxes.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_silu, silu.data(), SILU_BYTES, hipMemcpyHostToDevice);
  for (int o = 0; o < cfg->num_objects && e == hipSuccess; ++o) {
    const tg_sdf_grid& g = cfg->grids[o];
    e = hipMemcpy(h->d_vals + boxes[o].grid.offset, g.values, sizeof(float) * (size_t)g.n * g.n * g.n,
                  hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    tg_nsdf_destroy(h);
    return nfail(nullptr, TG_ERR_HIP, std::string("upload: ") + hipGetErrorString(e));
  }
  *out = h;
  return TG_OK;
}

tg_status tg_nsdf_destroy(tg_nsdf* h) {
  if (!h) return TG_OK;
  if (h->d_boxes) (void)hipFree(h->d_boxes);
  if (h->d_vals) (void)hipFree(h->d_vals);
  if (h->d_img) (void)hipFree(h->d_img);
  if (h->d_silu) (void)hipFree(h->d_silu);
  delete h;
  return TG_OK;
}

const char* tg_nsdf_last_error(const tg_nsdf* h) { return h ? h->err.c_str() : g_nsdf_create_error.c_str(); }

tg_status tg_nsdf_targets(tg_nsdf* h, const float* points, int64_t n, float* samples, float* grad_samples,
                          void* stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  if (!points || !samples || n < 1) return nfail(h, TG_ERR_INVALID_ARGUMENT, "targets: null pointer or n < 1");
  if (!aligned16(samples) || (grad_samples && !aligned16(grad_samples)))
    return nfail(h, TG_ERR_INVALID_ARGUMENT, "targets: samples not 16-byte aligned");
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)h->n_obj);
  hipLaunchKernelGGL(nsdf_targets_kernel, grid, dim3(256), 0, (hipStream_t)stream, h->d_boxes, h->d_vals, points, n,
                     (float4*)samples, (float4*)grad_samples);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? TG_OK : nfail(h, TG_ERR_HIP, hipGetErrorString(e));
}


tg_status tg_nsdf_grad(tg_nsdf* h, const float* params, const float* samples, const float* grad_samples, int64_t n,
                       float pair_lambda, float grad_lambda, float* grad, float* loss, void* stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  if (!params || !samples || !grad || n < 1) return nfail(h, TG_ERR_INVALID_ARGUMENT, "grad: null pointer or n < 1");
  if (const char* m = loss_terms_error(n, pair_lambda, grad_lambda, samples, grad_samples))
    return nfail(h, TG_ERR_INVALID_ARGUMENT, std::string("grad: ") + m);
  FitArgs a{};
  a.P = const_cast<float*>(params);
  a.samples = (const float4*)samples;
  a.n = n;
  a.grad = grad;
  a.loss = loss;
  a.n_obj = h->n_obj;
  a.pair_lambda = pair_lambda;
  a.gsamples = (const float4*)grad_samples;
  a.grad_lambda = grad_lambda;
  a.silu = h->d_silu;
  return grad_lambda > 0.f ? launch_fit<0, 1>(h, a, (hipStream_t)stream) : launch_fit<0, 0>(h, a, (hipStream_t)stream);
}

tg_status tg_nsdf_adam(float* params, float* m, float* v, const float* grad, int64_t count, int64_t t,
                       const tg_nsdf_train_params* hp, void* stream) {
  if (!params || !m || !v || !grad || !hp || count < 1 || t < 1) return TG_ERR_INVALID_ARGUMENT;
  const float c1 = (float)(1.0 - std::pow((double)hp->beta1, (double)t));
  const float c2 = (float)(1.0 - std::pow((double)hp->beta2, (double)t));
  hipLaunchKernelGGL(nsdf_adam_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     params, m, v, grad, count, hp->lr, hp->beta1, hp->beta2, hp->eps, c1, c2);
  return hipGetLastError() == hipSuccess ? TG_OK : TG_ERR_HIP;
}

tg_status tg_nsdf_train(tg_nsdf* h, float* params, float* m, float* v, const float* samples, const float* grad_samples,
                        int64_t n, int64_t step0, int32_t n_steps, const tg_nsdf_train_params* hp, float* loss,
                        void* stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  if (!params || !m || !v || !samples || !hp) return nfail(h, TG_ERR_INVALID_ARGUMENT, "train: null pointer");
  if (n < 1 || n > 0xffffffffLL || step0 < 0 || n_steps < 1 || step0 + n_steps > 0xffffffffLL)
    return nfail(h, TG_ERR_INVALID_ARGUMENT, "train: bad n / step range");
  if (hp->batch < 64 || hp->batch % 64) return nfail(h, TG_ERR_INVALID_ARGUMENT, "train: batch must be a multiple of 64");
  if (const char* msg = loss_terms_error(n, hp->pair_lambda, hp->grad_lambda, samples, grad_samples))
    return nfail(h, TG_ERR_INVALID_ARGUMENT, std::string("train: ") + msg);
  FitArgs a{};
  a.P = params;
  a.M = m;
  a.V = v;
  a.samples = (const float4*)samples;
  a.n = n;
  a.loss = loss;
  a.step0 = step0;
  a.n_steps = n_steps;
  a.n_obj = h->n_obj;
  a.batch = hp->batch;
  a.lr = hp->lr;
  a.b1 = hp->beta1;
  a.b2 = hp->beta2;
  a.eps = hp->eps;
  a.key0 = (uint32_t)hp->seed;
  a.key1 = (uint32_t)(hp->seed >> 32);
  a.pair_lambda = hp->pair_lambda;
  a.gsamples = (const float4*)grad_samples;
  a.grad_lambda = hp->grad_lambda;
  a.silu = h->d_silu;
  return hp->grad_lambda > 0.f ? launch_fit<1, 1>(h, a, (hipStream_t)stream)
                               : launch_fit<1, 0>(h, a, (hipStream_t)stream);
}

tg_status tg_nsdf_query(tg_nsdf* h, const float* params, const int64_t* offsets, int64_t max_count,
                        const float* xhat, float* out, float* grad, void* stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  if (!params || !offsets || !out || !xhat) return nfail(h, TG_ERR_INVALID_ARGUMENT, "query: null pointer");
  if (max_count < 0) return nfail(h, TG_ERR_INVALID_ARGUMENT, "query: max_count < 0");
  return launch_query(h, h->d_img, params, offsets, max_count, xhat, out, grad, (hipStream_t)stream);
}

tg_status tg_nsdf_query_trace(tg_nsdf* h, const float* params, const int64_t* offsets, int64_t max_count,
                              const float* xhat, float* out, float* grad, uint16_t* trace, void* stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  if (!params || !offsets || !out || !xhat || !trace)
    return nfail(h, TG_ERR_INVALID_ARGUMENT, "query_trace: null pointer");
  if (max_count < 0) return nfail(h, TG_ERR_INVALID_ARGUMENT, "query_trace: max_count < 0");
  return launch_query(h, h->d_img, params, offsets, max_count, xhat, out, grad, (hipStream_t)stream, trace);
}

tg_status tg_nsdf_query_noalloc(tg_nsdf* h, const float* params, const int64_t* offsets, int64_t max_count,
                                const float* xhat, float* out, float* grad, void* stream) {
  if (!h) return TG_ERR_INVALID_ARGUMENT;
  if (!params || !offsets || !out || !xhat) return nfail(h, TG_ERR_INVALID_ARGUMENT, "query_noalloc: null pointer");
  if (max_count < 0) return nfail(h, TG_ERR_INVALID_ARGUMENT, "query_noalloc: max_count < 0");
  if (h->n_obj > TG_NSDF_QUERY_NOALLOC_MAX_OBJECTS)
    return nfail(h, TG_ERR_INVALID_ARGUMENT,
                 "query_noalloc: " + std::to_string(h->n_obj) + " objects exceed the static scratch, which holds " +
                     std::to_string(TG_NSDF_QUERY_NOALLOC_MAX_OBJECTS) + " (use tg_nsdf_query)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return nfail(h, TG_ERR_HIP, "query_noalloc: hipGetDevice failed");
  if (dev != h->device)
    return nfail(h, TG_ERR_INVALID_ARGUMENT, "query_noalloc: the current device is not the handle's device");
  uint32_t* img = nullptr;
  const tg_status st = scratch_addr(h, dev, &img);
  if (st != TG_OK) return st;
  return launch_query(h, img, params, offsets, max_count, xhat, out, grad, (hipStream_t)stream);
}

}  // extern "C"
