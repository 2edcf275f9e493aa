// Device-side building blocks of the tactile readout (gfx950).
//
// The clean readout is one fixed FP32 operation sequence: every multiply-add
// that is fused is written as fmaf(), contraction is disabled for the whole
// build (-ffp-contract=off), division and sqrt are correctly rounded, and
// denormals are kept.  The same sequence gives the same bits on any IEEE FP32
// machine, which is what lets contact masks and depths be compared bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tg {

// A cubic SDF grid of n^3 samples.  The readout stores it in bricks of 4 x 4 x 4 values (256 B):
// sample (x, y, z) lives at offset + ((z/4 * nb + y/4) * nb + x/4) * 64 + (z%4 * 4 + y%4) * 4 + x%4,
// nb = ceil(n/4), so the 8 corners of a cell fall in one or two 128-byte lines and neighbouring
// probes of a patch share bricks.  (The training-target kernels keep plain x-fastest order, nb = 0.)
struct GridDesc {
  float origin[3];
  float spacing;
  float hinv;      // RN(1 / spacing), computed once on the host in FP32
  float nm1;       // (float)(n - 1)
  int32_t n;
  int32_t nb;      // bricks per axis
  int64_t offset;  // first value (a brick boundary) in the concatenated grid buffer
};

struct Pose {     // rotation, position, velocity, angular velocity
  float R[9];
  float p[3];
  float v[3];
  float w[3];
};

// Rotation matrix of a Hamilton quaternion (w,x,y,z), used as given.
__device__ __forceinline__ void quat_to_R(float w, float x, float y, float z, float* R) {
  const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  R[0] = 1.0f - 2.0f * (yy + zz);
  R[1] = 2.0f * (xy - wz);
  R[2] = 2.0f * (xz + wy);
  R[3] = 2.0f * (xy + wz);
  R[4] = 1.0f - 2.0f * (xx + zz);
  R[5] = 2.0f * (yz - wx);
  R[6] = 2.0f * (xz - wy);
  R[7] = 2.0f * (yz + wx);
  R[8] = 1.0f - 2.0f * (xx + yy);
}

// y = R x with rows as fma(R_i2, x2, fma(R_i1, x1, R_i0 * x0))
__device__ __forceinline__ void mat_vec(const float* R, float x0, float x1, float x2, float* y) {
#pragma unroll
  for (int i = 0; i < 3; ++i) y[i] = fmaf(R[3 * i + 2], x2, fmaf(R[3 * i + 1], x1, R[3 * i] * x0));
}
// y = R^T x
__device__ __forceinline__ void mat_T_vec(const float* R, float x0, float x1, float x2, float* y) {
#pragma unroll
  for (int i = 0; i < 3; ++i) y[i] = fmaf(R[6 + i], x2, fmaf(R[3 + i], x1, R[i] * x0));
}
__device__ __forceinline__ void cross3(const float* a, const float* b, float* c) {
  c[0] = fmaf(a[1], b[2], -(a[2] * b[1]));
  c[1] = fmaf(a[2], b[0], -(a[0] * b[2]));
  c[2] = fmaf(a[0], b[1], -(a[1] * b[0]));
}
__device__ __forceinline__ float lerpf(float t, float a, float b) { return fmaf(t, b - a, a); }

// ---------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds, two 32x32->64 products per round, key bumped
// by the Weyl constants between rounds.
// ---------------------------------------------------------------------------------------------
// a ^ b ^ k in one v_bitop3_b32 (truth table 0x96 = three-way xor; k uniform, in an SGPR)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                              uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = xor3(hi1, c1, k0);
    const uint32_t n2 = xor3(hi0, c3, k1);
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Uniform in (0,1) from the top 23 bits: (2*(x>>9)+1) * 2^-24, exact in FP32.
__device__ __forceinline__ float u01(uint32_t x) { return (float)(2u * (x >> 9) + 1u) * 5.9604644775390625e-08f; }

// Box-Muller pair from two uniforms; hardware log2 / sqrt / sin / cos (turn-based arguments).
__device__ __forceinline__ void box_muller(uint32_t xa, uint32_t xb, float& g0, float& g1) {
  const float ua = u01(xa), ub = u01(xb);
  const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(ua));
  g0 = r * __builtin_amdgcn_cosf(ub);
  g1 = r * __builtin_amdgcn_sinf(ub);
}

// Gaussian stream layout (purpose base p0: 0 = drift, 2 = white noise), per (env, taxel, t):
//   Philox(env, taxel, t, p0)        -> Box-Muller (x0,x1) -> ch0, ch1; (x2,x3) -> ch2, ch3
//   Philox(env, taxel, t >> 1, p0+1) -> even t: (y0,y1) -> ch4, ch5; odd t: (y2,y3) -> ch4, ch5
// The second call serves two consecutive steps; its second pair can be carried over.
__device__ __forceinline__ void gauss4(uint32_t k0, uint32_t k1, uint32_t env, uint32_t taxel, uint32_t t,
                                       uint32_t p0, float* g) {
  uint32_t x0 = env, x1 = taxel, x2 = t, x3 = p0;
  philox4x32_10(x0, x1, x2, x3, k0, k1);
  box_muller(x0, x1, g[0], g[1]);
  box_muller(x2, x3, g[2], g[3]);
}
__device__ __forceinline__ void pair_call(uint32_t k0, uint32_t k1, uint32_t env, uint32_t taxel, uint32_t tpair,
                                          uint32_t p0, uint32_t& y0, uint32_t& y1, uint32_t& y2, uint32_t& y3) {
  y0 = env; y1 = taxel; y2 = tpair; y3 = p0 + 1u;
  philox4x32_10(y0, y1, y2, y3, k0, k1);
}

// BF16 (round to nearest even) of a finite FP32 value, as the 16-bit pattern.
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

}  // namespace tg
