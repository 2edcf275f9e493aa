// Dense per-link spatial crosstalk on MFMA (App. A, KinematicTaxel / Sensor Noise Model:
// z~ = (1 - chi) z + chi (G_sigma * z), written as a matrix C_l = (1-chi) I + chi G_l on the
// uneven taxel set of each link, G_l the row-L1-normalised Gaussian of link-frame distances).
//
// For a block of `envs` envs of one link the six F/T channels of every env form the columns
// of Z_l (n_l x 6*envs); the block computes C_l Z_l with v_mfma_f32_16x16x32_bf16 (BF16
// operands, FP32 accumulation).  C_l is rounded once on the host (FP64 -> FP32 -> BF16, ties to even)
// and stored as ready-made A fragments; Z is rounded to BF16 by the lanes that own it and
// staged in LDS with every link padded to a multiple of 32 K rows (padding stays zero).
//
// MFMA 16x16x32 (bf16) lane layout, 64 lanes = 4 groups g of 16, 8 K slots per lane.  A and B
// must give slot (g, j) the same K index, and nothing else is required of the mapping; here slot
// (g, j) of K tile kt is k = 32 kt + 8 g + j, so a lane's B items are 8 consecutive bf16 of one
// staged column (one 16-byte LDS read):
//   A: lane i holds A[i%16][32 kt + 8 (i/16) + j]        j = 0..7
//   B: lane i holds B[32 kt + 8 (i/16) + j][i%16]
//   D: lane i holds D[4 (i/16) + r][i%16]                r = 0..3
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tg_readout.h"
#include "readout_kernel.h"

namespace tg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct XtDense {
  uint4* afrag = nullptr;     // per link: [mt][kt][64 lanes] x 8 bf16 (K tiles of 32)
  std::vector<void*> allocs;
};

inline uint16_t host_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Build C_l for every link in FP64, round once (FP64 -> FP32 -> BF16, ties to even) and lay
// the blocks out as MFMA A fragments.  Fills mt/kt/afrag_off of `links`.
inline tg_status xt_dense_setup(XtDense& X, const tg_readout_config* cfg, LinkInfo* links, std::string* err) {
  const int L = cfg->num_links;
  const int32_t* off = cfg->link_taxel_offset;
  const double chi = (double)cfg->noise.xtalk_chi, sg = (double)cfg->noise.xtalk_sigma;
  std::vector<uint4> frag;
  for (int l = 0; l < L; ++l) {
    const int a = off[l], n = off[l + 1] - a;
    const int MT = (n + 15) / 16, KT = (n + 31) / 32;
    links[l].mt = MT;
    links[l].kt = KT;
    links[l].afrag_off = (int32_t)(frag.size() / 64);
    if (n == 0) continue;
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
    for (int mt = 0; mt < MT; ++mt)
      for (int kt = 0; kt < KT; ++kt)
        for (int lane = 0; lane < 64; ++lane) {
          uint16_t v[8];
          for (int j = 0; j < 8; ++j) {
            const int m = 16 * mt + lane % 16, k = 32 * kt + 8 * (lane / 16) + j;
            v[j] = (m < n && k < n) ? host_bf16((float)C[(size_t)m * n + k]) : (uint16_t)0;
          }
          frag.push_back(make_uint4((uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16),
                                    (uint32_t)v[4] | ((uint32_t)v[5] << 16), (uint32_t)v[6] | ((uint32_t)v[7] << 16)));
        }
  }
  hipError_t e = hipMalloc(&X.afrag, std::max<size_t>(frag.size(), 1) * sizeof(uint4));
  if (e == hipSuccess) X.allocs.push_back(X.afrag);
  if (e == hipSuccess && !frag.empty())
    e = hipMemcpy(X.afrag, frag.data(), frag.size() * sizeof(uint4), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    *err = std::string("dense crosstalk setup: ") + hipGetErrorString(e);
    return TG_ERR_OUT_OF_MEMORY;
  }
  return TG_OK;
}

}  // namespace tg
