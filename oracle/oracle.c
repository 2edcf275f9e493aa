/* CPU oracle for the tactile readout.  TEST INFRASTRUCTURE ONLY: it is called
 * by the tests, by the package smoke check and by the CPU-baseline leg of the
 * benchmark, never by the product path.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * Contraction must stay off: the FP32 build is the written operation sequence,
 * with every fused multiply-add spelled out as fmaf().
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies; the key is bumped
 * by the Weyl constants before every round but the first. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* u in (0,1): the top 23 bits of x, centred in their cell, (2*(x>>9)+1) * 2^-24.
 * Exact in both FP32 and FP64. */
static double or_u01(uint32_t x) { return (double)(2u * (x >> 9) + 1u) * (1.0 / 16777216.0); }

/* Round an FP32 value to the nearest BF16 (ties to even), returned as FP32. */
float or_bf16_round(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) {
    if (u & 0x007fffffu) u |= 0x00400000u;
    u &= 0xffff0000u;
  } else {
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
  }
  memcpy(&x, &u, 4);
  return x;
}

/* Dense per-link crosstalk operator (App. A, spatial crosstalk, written as a
 * matrix on uneven patches): C_l = (1-chi) I + chi G_l, with G_l the Gaussian of
 * link-frame taxel distances at std sigma, each row L1-normalised. */
int or_dense_xtalk_f64(const or_problem* P, double* out) {
  const double chi = (double)P->xtalk_chi, sg = (double)P->xtalk_sigma;
  int64_t off = 0;
  for (int l = 0; l < P->num_links; ++l) {
    const int a = P->link_offset[l], n = P->link_offset[l + 1] - a;
    for (int r = 0; r < n; ++r) {
      double* row = out + off + (int64_t)r * n;
      double sum = 0;
      for (int c = 0; c < n; ++c) {
        double d2 = 0;
        for (int i = 0; i < 3; ++i) {
          double dx = (double)P->taxel_pos[3 * (a + r) + i] - (double)P->taxel_pos[3 * (a + c) + i];
          d2 += dx * dx;
        }
        row[c] = exp(-d2 / (2.0 * sg * sg));
        sum += row[c];
      }
      for (int c = 0; c < n; ++c) row[c] = chi * row[c] / sum + (r == c ? 1.0 - chi : 0.0);
    }
    off += (int64_t)n * n;
  }
  return 0;
}

#define REAL float
#define SFX(name) name##_f32
#define FMA fmaf
#define SQRT sqrtf
#define FLOOR floorf
#define POW powf
#define RINT rintf
#define FABS fabsf
#include "oracle_impl.h"
#undef REAL
#undef SFX
#undef FMA
#undef SQRT
#undef FLOOR
#undef POW
#undef RINT
#undef FABS

#define REAL double
#define SFX(name) name##_f64
#define FMA fma
#define SQRT sqrt
#define FLOOR floor
#define POW pow
#define RINT rint
#define FABS fabs
#include "oracle_impl.h"
