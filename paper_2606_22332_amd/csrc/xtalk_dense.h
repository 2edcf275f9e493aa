// Dense per-link spatial crosstalk on MFMA (App. A, KinematicTaxel / Sensor Noise Model:
// z~ = (1 - chi) z + chi (G_sigma * z), written as a matrix C_l = (1-chi) I + chi G_l on the
// uneven taxel set of each link, G_l the row-L1-normalised Gaussian of link-frame distances).
//
// For a block of `eb` envs the six F/T channels of every env form the columns of
// Z_l (n_l x 6*eb); the block computes C_l Z_l with v_mfma_f32_16x16x16_bf16 (BF16 operands,
// FP32 accumulation).  C_l is rounded once on the host (FP64 -> FP32 -> BF16, ties to even)
// and stored as ready-made A fragments; Z is rounded to BF16 by the lanes that own it and
// staged in LDS with every link padded to a multiple of 16 rows (padding stays zero).
//
// MFMA 16x16x16 (bf16, "1k") lane layout, 64 lanes, 4 elements per lane:
//   A: lane i holds A[i%16][4*(i/16) + r]        r = 0..3
//   B: lane i holds B[4*(i/16) + r][i%16]
//   D: lane i holds D[4*(i/16) + r][i%16]
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tg_readout.h"
#include "readout_kernel.h"

namespace tg {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct XtDense {
  uint2* afrag = nullptr;     // [tiles][64] lanes x 4 bf16
  int4* items = nullptr;      // (link, mtile, ntile, first A tile of (mtile, kt=0))
  int32_t* poff = nullptr;    // [L] padded offset of each link
  int32_t n_items = 0;
  int32_t tpad = 0;
  std::vector<void*> allocs;
};

inline uint16_t host_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Build C_l, the A fragments and the work items.  Returns TG_OK or an error with *err set.
inline tg_status xt_dense_setup(XtDense& X, const tg_readout_config* cfg, int eb, std::string* err) {
  const int L = cfg->num_links;
  const int32_t* off = cfg->link_taxel_offset;
  const double chi = (double)cfg->noise.xtalk_chi, sg = (double)cfg->noise.xtalk_sigma;
  std::vector<int32_t> poff(L);
  int tpad = 0;
  for (int l = 0; l < L; ++l) {
    poff[l] = tpad;
    tpad += ((off[l + 1] - off[l] + 15) / 16) * 16;
  }
  const int ncols = 6 * eb, ntiles = (ncols + 15) / 16;
  std::vector<uint2> frag;
  std::vector<int4> items;
  for (int l = 0; l < L; ++l) {
    const int a = off[l], n = off[l + 1] - a;
    if (n == 0) continue;
    // C_l in FP64
    std::vector<double> C((size_t)n * n);
    for (int r = 0; r < n; ++r) {
      double sum = 0;
      for (int c = 0; c < n; ++c) {
        double d2 = 0;
        for (int i = 0; i < 3; ++i) {
          const double dx = (double)cfg->taxel_pos[3 * (a + r) + i] - (double)cfg->taxel_pos[3 * (a + c) + i];
          d2 += dx * dx;
        }
        C[(size_t)r * n + c] = std::exp(-d2 / (2.0 * sg * sg));
        sum += C[(size_t)r * n + c];
      }
      for (int c = 0; c < n; ++c) C[(size_t)r * n + c] = chi * C[(size_t)r * n + c] / sum + (r == c ? 1.0 - chi : 0.0);
    }
    const int MT = (n + 15) / 16, KT = MT;
    const int first = (int)(frag.size() / 64);
    for (int mt = 0; mt < MT; ++mt)
      for (int kt = 0; kt < KT; ++kt)
        for (int lane = 0; lane < 64; ++lane) {
          uint16_t v[4];
          for (int r = 0; r < 4; ++r) {
            const int m = 16 * mt + lane % 16, k = 16 * kt + 4 * (lane / 16) + r;
            v[r] = (m < n && k < n) ? host_bf16((float)C[(size_t)m * n + k]) : (uint16_t)0;
          }
          frag.push_back(make_uint2((uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16)));
        }
    for (int mt = 0; mt < MT; ++mt)
      for (int nt = 0; nt < ntiles; ++nt) items.push_back(make_int4(l, mt, nt, first + mt * KT));
  }
  hipError_t e = hipMalloc(&X.afrag, std::max<size_t>(frag.size(), 1) * sizeof(uint2));
  if (e == hipSuccess) X.allocs.push_back(X.afrag);
  if (e == hipSuccess) e = hipMalloc(&X.items, std::max<size_t>(items.size(), 1) * sizeof(int4));
  if (e == hipSuccess) X.allocs.push_back(X.items);
  if (e == hipSuccess) e = hipMalloc(&X.poff, L * sizeof(int32_t));
  if (e == hipSuccess) X.allocs.push_back(X.poff);
  if (e == hipSuccess) e = hipMemcpy(X.afrag, frag.data(), frag.size() * sizeof(uint2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(X.items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(X.poff, poff.data(), L * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    *err = std::string("dense crosstalk setup: ") + hipGetErrorString(e);
    return TG_ERR_OUT_OF_MEMORY;
  }
  X.n_items = (int32_t)items.size();
  X.tpad = tpad;
  return TG_OK;
}

// Block-wide dense crosstalk: z (this lane's six channels after gain) -> zt.  Every thread of
// the block must call it (it holds two barriers).  xtb: [6][eb][tpad] bf16 staging (padding
// rows zero), xtx: [6][eb][tpad] fp32 results.
__device__ __forceinline__ void xtalk_dense_block(const KParams& p, const float* z, float* zt,
                                                  unsigned char* xtb_raw, unsigned char* xtx_raw, int el, int j,
                                                  int lk, bool act, int e0) {
  (void)e0;
  uint16_t* xb = (uint16_t*)xtb_raw;
  float* xx = (float*)xtx_raw;
  const int eb = p.eb, tpad = p.tpad;
  int row = 0;
  if (act) {
    row = p.xt_poff[lk] + (j - p.link_off[lk]);
#pragma unroll
    for (int c = 0; c < 6; ++c) xb[(size_t)(c * eb + el) * tpad + row] = (uint16_t)bf16_bits(z[c]);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int it = wave; it < p.xt_n_items; it += nwaves) {
    const int4 item = p.xt_items[it];   // (link, mtile, ntile, first A tile)
    const int l = item.x, mt = item.y, nt = item.z;
    const int nl = p.link_off[l + 1] - p.link_off[l];
    const int KT = (nl + 15) >> 4;
    const int n = nt * 16 + (lane & 15);
    const bool colok = n < 6 * eb;
    const int c = n % 6, elc = n / 6;
    const uint16_t* bcol = xb + (size_t)(c * eb + elc) * tpad + p.xt_poff[l] + 4 * (lane >> 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < KT; ++kt) {
      const uint2 a = p.xt_afrag[(size_t)(item.w + kt) * 64 + lane];
      const uint2 b = colok ? *(const uint2*)(bcol + 16 * kt) : make_uint2(0u, 0u);
      bf16x4 av, bv;
      __builtin_memcpy(&av, &a, 8);
      __builtin_memcpy(&bv, &b, 8);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
    if (colok) {
      const int m0 = 16 * mt + 4 * (lane >> 4);
      float* dst = xx + (size_t)(c * eb + elc) * tpad + p.xt_poff[l];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (m0 + r < nl) dst[m0 + r] = acc[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 6; ++c) zt[c] = act ? xx[(size_t)(c * eb + el) * tpad + row] : 0.f;
}

}  // namespace tg
