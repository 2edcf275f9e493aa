/* tg_audio — the contact-audio sensor (App. E, contact audio) on one MI355X (gfx950).
 *
 * Source-filter modal synthesis: a material is a bank of damped two-pole resonators, and the
 * contacts of a sensor link excite it.  Each physics step of length dt emits K samples at
 * dt_sub = dt / K (sample rate K / dt).  Mode i of a material, (f_i, d_i, g_i) = (frequency [Hz],
 * decay rate [1/s], output gain), advances as
 *   y_i[k] = a1_i y_i[k-1] - a2_i y_i[k-2] + u[k],  a1_i = 2 r_i cos(2 pi f_i dt_sub),
 *   a2_i = r_i^2,  r_i = exp(-d_i dt_sub),
 * and the sample is s[k] = sum_i g_i y_i[k].  The excitation of sensor link l in env e at step t is
 * read from the readout's taxel forces f_j and contact normals m_j (link frame):
 *   F_n = sum_{j in l} f_j . m_j                     (normal force of the kinematic law)
 *   F_t = sum_{j in l} |f_j - (f_j . m_j) m_j|       (its friction, scaled by slip and capped)
 *   u[0] += g_imp max(0, F_n(t) - F_n(t-1))          (impact: a rise of the normal force)
 *   u[k] += g_scr F_t xi[k],  k = 0..K-1             (scrape: friction-scaled noise)
 * xi[k] = 2 u - 1, u = (2 (w >> 9) + 1) 2^-24, w = word k mod 4 of Philox4x32-10 with key = seed and
 * counter (env, 2^31 + l, t, k / 4): uniform on (-1, 1) and exact in FP32.
 *
 * The bank has `slots` slots; a material with fewer modes fills the rest with silent slots
 * (a1 = a2 = g = 0), and an env whose material id is out of range has every slot silent.  The
 * resonator states and the previous F_n of every (env, sensor link) live in the handle and carry
 * over from call to call (tg_audio_reset zeroes them).  The resonators and the excitation run in
 * FP64 (the MI355X vector FP64 rate equals its unpacked FP32 rate); each sample is rounded once to
 * FP32 on output.  The coefficients a1, a2 are formed on the host in FP64 at create.
 *
 * Conventions are those of tg_readout.h: create deep-copies the host arrays; device buffers are
 * caller-owned and must stay valid until the queued work finishes; calls return a tg_status and
 * launch nothing on error; rollout allocates nothing and never synchronises.  Calls on one handle
 * must not overlap (they share its state).
 */
#ifndef TG_AUDIO_H
#define TG_AUDIO_H
#include <stddef.h>
#include <stdint.h>

#include "tg_readout.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tg_audio tg_audio; /* opaque: coefficient table and resonator state on the device */

typedef struct {
  int32_t num_modes;     /* >= 0, <= slots */
  const double* freq;    /* host [num_modes] f_i [Hz], finite, >= 0 */
  const double* decay;   /* host [num_modes] d_i [1/s], finite, >= 0 */
  const double* gain;    /* host [num_modes] g_i, finite */
} tg_audio_material;

typedef struct {
  uint32_t abi_version;               /* TG_ABI_VERSION */
  int32_t num_envs;                   /* E >= 1 */
  int32_t num_taxels;                 /* T: row length of the readout's ft / normal planes */
  int32_t num_sensor_links;           /* Ls >= 1 */
  const int32_t* sensor_taxel_begin;  /* host [Ls] first taxel of each sensor link */
  const int32_t* sensor_taxel_end;    /* host [Ls] one past its last; 0 <= begin <= end <= T */
  int32_t num_materials;              /* >= 0 */
  const tg_audio_material* materials; /* host [num_materials] */
  int32_t slots;                      /* bank slots, 1..32 (rounded up to 4, 8, 16 or 32) */
  int32_t samples_per_step;           /* K, 1..1024 */
  double dt;                          /* physics step [s], > 0 */
  double g_imp, g_scr;                /* impact and scrape gains, finite */
  uint64_t seed;                      /* Philox key of the scrape noise */
  int32_t lanes_per_pair;             /* lanes sharing one (env, link) bank: 1, 2, 4, 8 or 16, or 0 =
                                         chosen at create (the smallest giving every SIMD two
                                         waves, else the largest whose block fits in LDS) */
} tg_audio_config;

/* TG_ERR_INVALID_ARGUMENT for sizes or values outside the ranges above or NULL arrays;
 * TG_ERR_UNSUPPORTED when E * T * 6 does not fit 32 bits. */
tg_status tg_audio_create(const tg_audio_config* cfg, tg_audio** out);

/* n_steps consecutive steps in one launch, the first with step index step0 (noise counter).
 * ft: device [n_steps][6][E][T] taxel force/torque (only the forces are read), normal: device
 * [n_steps][3][E][T] contact normals (0 where there is no contact), as tg_readout writes them;
 * material: device [E] bank index per env; out: device [n_steps][E][Ls][K].
 * Pointers 16-byte aligned; step0 + n_steps <= 2^32. */
tg_status tg_audio_rollout(tg_audio* h, const float* ft, const float* normal, const int32_t* material,
                           int64_t step0, int32_t n_steps, float* out, void* hip_stream);

/* Zeroes the resonator states and the previous normal forces (a small fill kernel on the
 * stream, no memset node, so the call may be captured). */
tg_status tg_audio_reset(tg_audio* h, void* hip_stream);

tg_status tg_audio_destroy(tg_audio* h); /* NULL is OK */
const char* tg_audio_last_error(const tg_audio* h);

#ifdef __cplusplus
}
#endif
#endif /* TG_AUDIO_H */
