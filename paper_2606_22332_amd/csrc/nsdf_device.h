// Neural signed-distance surrogate on gfx950 MFMA: device building blocks.
//
// Network per object: x_hat in [-1,1]^3 (the object's grid box mapped to the unit cube)
//   -> positional encoding sin/cos(2^k pi x_hat_d), k = 0..7 (48 features)
//   -> 4 hidden layers of width 64, SiLU -> 1 linear output; phi = half_extent * out.
// Flat FP32 parameter order: W1[64][48], b1[64], W2[64][64], b2, W3, b3, W4, b4, w5[64], b5.
//
// MFMA layout (v_mfma_f32_16x16x32_bf16, one wave = 16 samples = one "tile").  The accumulator of
// a 16x16 product gives lane i = 16g + s the rows 4g+r (r = 0..3) of column s.  A layer computes
// Z[out][sample] = W[out][in] * A[in][sample], so after a layer lane (g, s) holds, for sample s,
// the outputs 16m + 4g + r of each M-tile m.  The next layer's B operand for K-tile kt takes its
// eight K-items from M-tiles 2kt and 2kt+1 unchanged, which fixes the K order
//   item r of lane group g  <->  feature 32kt + 16(r/4) + 4g + r%4.
// The weights are packed in that K order once (pack kernel or in-block repack), so activations
// never leave registers between layers.  A and B of an MFMA share the item -> K mapping, which
// is all the contraction needs.
//
// The first layer's input is the positional encoding.  Its internal K order is chosen so that
// lane group g of K-tile kt evaluates one frequency k = 4kt + g: items 0..2 = sin of x, y, z,
// items 3..5 = cos, items 6..7 = zero padding (48 real features in 64 K slots).
//
// Packed per-object image (IMG_BYTES):
//   [0, 32768)      forward A fragments, (layer, m-tile, k-tile) -> 1 KiB = 64 lanes x 8 bf16
//   [32768, 63488)  transposed A fragments for the reverse pass (rows = layer inputs,
//                   K = layer outputs in chain order); layer 1 has 3 row tiles (48 inputs)
//   [63488, 65024)  FP32 tail: b1..b4 at 64*l, w5 at 256, b5 at 320
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "readout_device.h"

namespace tg {
namespace nsdf {

constexpr int H = 64, F = 48, NPARAM = 15681;
constexpr int W_OFF[4] = {0, 3136, 7296, 11456};
constexpr int B_OFF[4] = {3072, 7232, 11392, 15552};
constexpr int W5_OFF = 15616, B5_OFF = 15680;
constexpr int FWD_BYTES = 32768, BWD_BYTES = 30720, TAIL_FLOATS = 384;
constexpr int IMG_BYTES = FWD_BYTES + BWD_BYTES + TAIL_FLOATS * 4;  // 65024
constexpr int IMG_WORDS = IMG_BYTES / 4;
// SiLU table: bf16(silu(z)) for every BF16 z with 2^-13 <= |z| < 2^7 (biased exponents
// 114..133), at entry (sign << 12) | ((exponent - 114) << 7) | mantissa: the negative half
// starts 4096 entries (8 KB) in, so that the sign bit becomes the offset with one shift;
// entries 2560..4095 are unused.  Outside that range the BF16 result has a closed
// form: z / 2 for smaller |z| (the z^2/4 term is below half an ulp), z itself for z >= 128 and
// -0 for z <= -128 (the product underflows FP32).  Kernels keep the table in a static LDS array
// (constant address, folded into the read's offset field).
constexpr int SILU_E0 = 114, SILU_NE = 20, SILU_NEG = 4096;
constexpr int SILU_ENTRIES = SILU_NEG + SILU_NE * 128;   // 6656
constexpr int SILU_BYTES = SILU_ENTRIES * 2;            // 13312

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short short4v __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mfma32(u32x4 a, u32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(u32x2 a, u32x2 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(short4v, a), __builtin_bit_cast(short4v, b),
                                                   c, 0, 0, 0);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// Two FP32 values rounded to BF16 (nearest even) and packed low, high: one v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){lo, hi}, bf16x2));
}
__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// logistic function from the hardware 2^x and reciprocal
__device__ __forceinline__ float sigmoid(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// ---------------------------------------------------------------------------------------------
// parameter <-> packed-image maps
// ---------------------------------------------------------------------------------------------
// chain K order inside a 32-wide K-tile: item (g, r) <-> 16(r/4) + 4g + r%4
__device__ __forceinline__ int chain_k(int g, int r) { return 16 * (r >> 2) + 4 * g + (r & 3); }

// Parameter index held by forward fragment (l, m, kt), lane, item r; -1 = zero padding.
__device__ __forceinline__ int fwd_param(int l, int m, int kt, int lane, int r) {
  const int o = 16 * m + (lane & 15), g = lane >> 4;
  if (l == 0) {
    if (r >= 6) return -1;
    return W_OFF[0] + o * F + 6 * (4 * kt + g) + r;
  }
  return W_OFF[l] + o * H + 32 * kt + chain_k(g, r);
}
// Reverse-pass fragment bi (layer 1: bi = 2m + kt, m < 3; layer l >= 2: 6 + ((l-1)*4 + m)*2 + kt).
__device__ __forceinline__ int bwd_param(int bi, int lane, int r) {
  int l, m, kt;
  if (bi < 6) { l = 0; m = bi >> 1; kt = bi & 1; }
  else { const int q = bi - 6; l = 1 + (q >> 3); m = (q >> 1) & 3; kt = q & 1; }
  const int in = 16 * m + (lane & 15), g = lane >> 4;
  const int o = 32 * kt + chain_k(g, r);
  return W_OFF[l] + o * (l == 0 ? F : H) + in;
}
// Value of 32-bit image word w of the image built from params P (FP32).
__device__ __forceinline__ uint32_t image_word(const float* P, int w) {
  if (w < FWD_BYTES / 4) {
    const int frag = w >> 8, lane = (w >> 2) & 63, q = w & 3;
    const int l = frag >> 3, m = (frag >> 1) & 3, kt = frag & 1;
    const int p0 = fwd_param(l, m, kt, lane, 2 * q), p1 = fwd_param(l, m, kt, lane, 2 * q + 1);
    return pack2(p0 < 0 ? 0.f : P[p0], p1 < 0 ? 0.f : P[p1]);
  }
  if (w < (FWD_BYTES + BWD_BYTES) / 4) {
    const int v = w - FWD_BYTES / 4;
    const int bi = v >> 8, lane = (v >> 2) & 63, q = v & 3;
    return pack2(P[bwd_param(bi, lane, 2 * q)], P[bwd_param(bi, lane, 2 * q + 1)]);
  }
  const int t = w - (FWD_BYTES + BWD_BYTES) / 4;
  float x = 0.f;
  if (t < 256) x = P[B_OFF[t >> 6] + (t & 63)];
  else if (t < 320) x = P[W5_OFF + t - 256];
  else if (t == 320) x = P[B5_OFF];
  return __float_as_uint(x);
}

// Byte offsets of a weight W_l[o][in] inside the image: forward and reverse copies.
__device__ __forceinline__ void weight_slots(int l, int o, int in, int& fwd_off, int& bwd_off) {
  const int m = o >> 4;
  int kt, g, r;
  if (l == 0) {
    const int k = in / 6;
    r = in - 6 * k;
    kt = k >> 2;
    g = k & 3;
  } else {
    kt = in >> 5;
    const int rem = in & 31;
    g = (rem & 15) >> 2;
    r = 4 * (rem >> 4) + (rem & 3);
  }
  fwd_off = (((l * 4 + m) * 2 + kt) << 10) + ((16 * g + (o & 15)) << 4) + 2 * r;
  const int mb = in >> 4, ktb = o >> 5, remb = o & 31;
  const int gb = (remb & 15) >> 2, rb = 4 * (remb >> 4) + (remb & 3);
  const int bi = l == 0 ? 2 * mb + ktb : 6 + ((l - 1) * 4 + mb) * 2 + ktb;
  bwd_off = FWD_BYTES + (bi << 10) + ((16 * gb + (in & 15)) << 4) + 2 * rb;
}

// ---------------------------------------------------------------------------------------------
// per-tile network evaluation (one wave, 16 samples; lane = 16g + s)
// ---------------------------------------------------------------------------------------------
struct Img {
  const uint8_t* fwd;
  const uint8_t* bwd;
  const float* tail;
};
__device__ __forceinline__ Img img_at(const uint8_t* base) {
  return Img{base, base + FWD_BYTES, (const float*)(base + FWD_BYTES + BWD_BYTES)};
}
__device__ __forceinline__ u32x4 frag(const uint8_t* base, int idx, int lane) {
  return *(const u32x4*)(base + (idx << 10) + (lane << 4));
}

// Positional-encoding B fragments.  sin(2^k pi x) = sin(2 pi * frac(2^(k-1) x)); the hardware
// sine and cosine take their argument in turns.
__device__ __forceinline__ void pe_frags(float x0, float x1, float x2, int g, u32x4 b[2]) {
#pragma unroll
  for (int kt = 0; kt < 2; ++kt) {
    const float sc = (float)(1 << (4 * kt + g)) * 0.5f;
    const float t0 = __builtin_amdgcn_fractf(sc * x0), t1 = __builtin_amdgcn_fractf(sc * x1),
                t2 = __builtin_amdgcn_fractf(sc * x2);
    const float s0 = __builtin_amdgcn_sinf(t0), s1 = __builtin_amdgcn_sinf(t1), s2 = __builtin_amdgcn_sinf(t2);
    const float c0 = __builtin_amdgcn_cosf(t0), c1 = __builtin_amdgcn_cosf(t1), c2 = __builtin_amdgcn_cosf(t2);
    b[kt] = u32x4{pack2(s0, s1), pack2(s2, c0), pack2(c1, c2), 0u};
  }
}

// One hidden layer: acc[m] = b + W * in (FP32 accumulation).
__device__ __forceinline__ void layer_fwd(const Img& im, int l, int lane, const u32x4 bin[2], f32x4 acc[4]) {
  const int g = lane >> 4;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    acc[m] = *(const f32x4*)(im.tail + 64 * l + 16 * m + 4 * g);
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) acc[m] = mfma32(frag(im.fwd, (l * 4 + m) * 2 + kt, lane), bin[kt], acc[m]);
  }
}

// Round the pre-activations to BF16 (kept in z), apply SiLU and form the next layer's B
// fragments; a4 receives the FP32 activations when the caller needs them (last layer).
__device__ __forceinline__ void activate(const f32x4 acc[4], uint32_t z[8], u32x4 bout[2], float a[4][4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    z[2 * m] = pack2(acc[m][0], acc[m][1]);
    z[2 * m + 1] = pack2(acc[m][2], acc[m][3]);
    const float zz[4] = {bf_lo(z[2 * m]), bf_hi(z[2 * m]), bf_lo(z[2 * m + 1]), bf_hi(z[2 * m + 1])};
#pragma unroll
    for (int r = 0; r < 4; ++r) a[m][r] = zz[r] * sigmoid(zz[r]);
  }
#pragma unroll
  for (int kt = 0; kt < 2; ++kt)
    bout[kt] = u32x4{pack2(a[2 * kt][0], a[2 * kt][1]), pack2(a[2 * kt][2], a[2 * kt][3]),
                     pack2(a[2 * kt + 1][0], a[2 * kt + 1][1]), pack2(a[2 * kt + 1][2], a[2 * kt + 1][3])};
}

// bf16(silu(z)) for the 16 BF16 pre-activations of a lane (4 packed words per pair of M-tiles,
// z[8]), from the table in LDS.  The table index of bits b is (b & 0x7fff) - 114*128 plus 4096
// for a negative sign; it is clamped into the table, and the rare values outside it (|z| < 2^-13
// or |z| >= 128) are fixed up afterwards on a wave-uniform branch with their closed forms.
__device__ __forceinline__ uint32_t silu_closed(uint32_t b) {
  const uint32_t t = (b & 0x7fffu) - (uint32_t)(SILU_E0 << 7);
  if ((int)t < 0) {   // |z| < 2^-13: z / 2
    const float half = __uint_as_float(b << 16) * 0.5f;
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){half, 0.f}, bf16x2)) & 0xffffu;
  }
  return (b >> 15) ? 0x8000u : b;   // |z| >= 128: z, or -0 below -128
}
__device__ __forceinline__ void silu_words(const uint32_t z[8], uint32_t out[8], const uint16_t* tab) {
  uint32_t v[16];
  bool any_out = false;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const uint32_t b = (i & 1) ? (z[i >> 1] >> 16) : (z[i >> 1] & 0xffffu);
    const uint32_t t = (b & 0x7fffu) - (uint32_t)(SILU_E0 << 7);
    any_out |= t >= (uint32_t)(SILU_NE << 7);
    const uint32_t idx = min(t, (uint32_t)(SILU_NE << 7) - 1u) + (b >> 15) * (uint32_t)SILU_NEG;
    v[i] = tab[idx];
  }
  if (__any(any_out)) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint32_t b = (i & 1) ? (z[i >> 1] >> 16) : (z[i >> 1] & 0xffffu);
      const uint32_t t = (b & 0x7fffu) - (uint32_t)(SILU_E0 << 7);
      if (t >= (uint32_t)(SILU_NE << 7)) v[i] = silu_closed(b);
    }
  }
#pragma unroll
  for (int w = 0; w < 8; ++w) out[w] = v[2 * w] | (v[2 * w + 1] << 16);
}

// Table path of a hidden layer: BF16 pre-activations (kept in z) and the next layer's BF16
// input fragments, without transcendentals.  Word w of z holds items (2w, 2w+1) of M-tile w/2.
__device__ __forceinline__ void activate_tab(const f32x4 acc[4], uint32_t z[8], u32x4 bout[2], const uint16_t* tab) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    z[2 * m] = pack2(acc[m][0], acc[m][1]);
    z[2 * m + 1] = pack2(acc[m][2], acc[m][3]);
  }
  uint32_t a[8];
  silu_words(z, a, tab);
#pragma unroll
  for (int kt = 0; kt < 2; ++kt) bout[kt] = u32x4{a[4 * kt], a[4 * kt + 1], a[4 * kt + 2], a[4 * kt + 3]};
}
__device__ __forceinline__ void act_frags_tab(const uint32_t z[8], u32x4 b[2], const uint16_t* tab) {
  uint32_t a[8];
  silu_words(z, a, tab);
#pragma unroll
  for (int kt = 0; kt < 2; ++kt) b[kt] = u32x4{a[4 * kt], a[4 * kt + 1], a[4 * kt + 2], a[4 * kt + 3]};
}

// Recompute a layer's BF16 input fragments from the stored BF16 pre-activations.
__device__ __forceinline__ void act_frags(const uint32_t z[8], u32x4 b[2]) {
  float a[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const float zz[4] = {bf_lo(z[2 * m]), bf_hi(z[2 * m]), bf_lo(z[2 * m + 1]), bf_hi(z[2 * m + 1])};
#pragma unroll
    for (int r = 0; r < 4; ++r) a[m][r] = zz[r] * sigmoid(zz[r]);
  }
#pragma unroll
  for (int kt = 0; kt < 2; ++kt)
    b[kt] = u32x4{pack2(a[2 * kt][0], a[2 * kt][1]), pack2(a[2 * kt][2], a[2 * kt][3]),
                  pack2(a[2 * kt + 1][0], a[2 * kt + 1][1]), pack2(a[2 * kt + 1][2], a[2 * kt + 1][3])};
}

// Sum over the four lane groups (lanes s, s+16, s+32, s+48).
__device__ __forceinline__ float group_sum(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// Forward pass of one tile.  Returns the network output for sample (lane & 15) on every lane;
// z receives the BF16 pre-activations of the four hidden layers, pe the input fragments.
__device__ __forceinline__ float forward_tile(const Img& im, int lane, float x0, float x1, float x2,
                                              uint32_t z[4][8], u32x4 pe[2], float a4[4][4], const uint16_t* tab) {
  const int g = lane >> 4;
  pe_frags(x0, x1, x2, g, pe);
  u32x4 b[2] = {pe[0], pe[1]};
  f32x4 acc[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    __builtin_amdgcn_sched_barrier(0);   // keep each layer's fragment loads next to its MFMAs
    layer_fwd(im, l, lane, b, acc);
    u32x4 nb[2];
    if (l < 3) {
      activate_tab(acc, z[l], nb, tab);   // layers 1-3 feed a BF16 GEMM: table SiLU
    } else {
      activate(acc, z[l], nb, a4);        // layer 4 feeds the FP32 output layer
    }
    b[0] = nb[0];
    b[1] = nb[1];
  }
  float part = 0.f;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) part = fmaf(im.tail[256 + 16 * m + 4 * g + r], a4[m][r], part);
  return group_sum(part) + im.tail[320];
}

// dz = g * silu'(z) for one layer, rounded to BF16 as B fragments (chain order).
__device__ __forceinline__ void dz_frags(const float g[4][4], const uint32_t z[8], u32x4 db[2], float dz[4][4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const float zz[4] = {bf_lo(z[2 * m]), bf_hi(z[2 * m]), bf_lo(z[2 * m + 1]), bf_hi(z[2 * m + 1])};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float sg = sigmoid(zz[r]);
      dz[m][r] = g[m][r] * (sg * fmaf(zz[r], 1.0f - sg, 1.0f));
    }
  }
#pragma unroll
  for (int kt = 0; kt < 2; ++kt)
    db[kt] = u32x4{pack2(dz[2 * kt][0], dz[2 * kt][1]), pack2(dz[2 * kt][2], dz[2 * kt][3]),
                   pack2(dz[2 * kt + 1][0], dz[2 * kt + 1][1]), pack2(dz[2 * kt + 1][2], dz[2 * kt + 1][3])};
}

// g_in = W_l^T dz over the layer's inputs (l >= 1: 4 row tiles; l == 0: 3 row tiles = 48 features).
template <int NM>
__device__ __forceinline__ void layer_bwd(const Img& im, int l, int lane, const u32x4 db[2], f32x4 out[NM]) {
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    out[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
      const int bi = l == 0 ? 2 * m + kt : 6 + ((l - 1) * 4 + m) * 2 + kt;
      out[m] = mfma32(frag(im.bwd, bi, lane), db[kt], out[m]);
    }
  }
}

// Gradient of the network output with respect to x_hat for sample (lane & 15), on every lane.
__device__ __forceinline__ void input_grad_tile(const Img& im, int lane, float x0, float x1, float x2,
                                                const uint32_t z[4][8], float gx[3]) {
  const int g = lane >> 4;
  float gr[4][4], dz[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) gr[m][r] = im.tail[256 + 16 * m + 4 * g + r];
#pragma unroll
  for (int l = 3; l >= 1; --l) {
    __builtin_amdgcn_sched_barrier(0);
    u32x4 db[2];
    dz_frags(gr, z[l], db, dz);
    f32x4 o[4];
    layer_bwd<4>(im, l, lane, db, o);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) gr[m][r] = o[m][r];
  }
  __builtin_amdgcn_sched_barrier(0);
  u32x4 db[2];
  dz_frags(gr, z[0], db, dz);
  f32x4 gf[3];
  layer_bwd<3>(im, 0, lane, db, gf);
  // feature f = 16m + 4g + r in the encoding's own order: f = 6k + 3c + d (c = 0 sine, 1 cosine)
  float p[3] = {0.f, 0.f, 0.f};
  const float xs[3] = {x0, x1, x2};
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = 16 * m + 4 * g + r;
      const int k = f / 6, rem = f - 6 * k, c = rem / 3, d = rem - 3 * c;
      const float sc = (float)(1 << k) * 0.5f;
      const float xd = d == 0 ? xs[0] : (d == 1 ? xs[1] : xs[2]);
      const float t = __builtin_amdgcn_fractf(sc * xd);
      const float w = (float)(1 << k) * 3.14159265358979323846f;
      const float dv = c == 0 ? w * __builtin_amdgcn_cosf(t) : -w * __builtin_amdgcn_sinf(t);
      const float contrib = gf[m][r] * dv;
      p[0] += d == 0 ? contrib : 0.f;
      p[1] += d == 1 ? contrib : 0.f;
      p[2] += d == 2 ? contrib : 0.f;
    }
  gx[0] = group_sum(p[0]);
  gx[1] = group_sum(p[1]);
  gx[2] = group_sum(p[2]);
}

// Host: the SiLU table, bf16(fp32(silu(z))) in FP64 with round to nearest even at both steps.
inline void build_silu_table(uint16_t* t) {
  for (int i = 0; i < SILU_ENTRIES; ++i) t[i] = 0;
  for (int sgn = 0; sgn < 2; ++sgn)
    for (int r = 0; r < SILU_NE; ++r)
      for (int m = 0; m < 128; ++m) {
        const uint32_t zb = ((uint32_t)sgn << 31) | ((uint32_t)(SILU_E0 + r) << 23) | ((uint32_t)m << 16);
        float zf;
        __builtin_memcpy(&zf, &zb, 4);
        const double z = zf;
        const float s = (float)(z / (1.0 + __builtin_exp(-z)));
        uint32_t u;
        __builtin_memcpy(&u, &s, 4);
        u += 0x7fffu + ((u >> 16) & 1u);
        t[sgn * SILU_NEG + ((r << 7) | m)] = (uint16_t)(u >> 16);
      }
}

}  // namespace nsdf
}  // namespace tg
