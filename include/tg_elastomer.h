/* tg_elastomer — the ElastomerTaxel (App. A.7) on one MI355X (gfx950).
 *
 * Marker displacements of a deformable pad on a sensor link, from SDF-driven dilation and
 * anchored shear history.  With Pi_n(z) = z - (z . n) n the projection onto a marker's tangent
 * plane, for marker j (link-frame position x_j, unit normal n_j) of a sensor link:
 *   dilation by each probe i of the same link, penetration h_i = max(0, d_i - R_i) from the
 *   readout's depth d_i = max(0, R_i - phi(q_i)) (so h_i = max(0, -phi(q_i))):
 *     r = Pi_{n_j}(x_j - x_i),  g = exp(-lambda_d |r|^2),  rho = 1 / (|r|^2 + eps^2),
 *     w = h_i (c g / g_bar + (1 - c) rho / rho_bar),  g_bar = e^{-1/2} / sqrt(2 lambda_d),
 *     rho_bar = 1 / (2 eps),   u^d = s_d (r w + n_j h_i^alpha g)
 *   shear by each tracked surface point p of the env's object (object-frame cloud, sensor-frame
 *   position z_p = R_L^T (R_O p_hat + p_O - p_L), pad SDF phi_e(z_p) = exact distance to the pad
 *   box, penetration h_p = max(0, -phi_e)):
 *     u^s = s_s Pi_{n_j}(z_p - e_p) h_p exp(-lambda_s |Pi_{n_j}(x_j - z_p)|^2)
 *   for points with an anchor e_p.  A point takes e_p = z_p when phi_e < -eta_enter and drops it
 *   when phi_e > eta_exit; anchors carry over between steps and calls, and a change of an env's
 *   object clears that env's anchors.  y_j = sum_i u^d + sum_p u^s.
 * The clamped-boundary correction of App. A.7 is not implemented (the configuration has none).
 *
 * The point positions, the pad SDF and the anchor decisions follow a fixed FP32 sequence
 * (fused multiply-adds written out, no other contraction, correctly rounded sqrt), so the
 * decisions are reproducible; the sums are FP32.
 *
 * Conventions are those of tg_readout.h: create deep-copies the host arrays; device buffers are
 * caller-owned and must stay valid until the queued work finishes; calls return a tg_status and
 * launch nothing on error; rollout allocates nothing and never synchronises.  Calls on one handle
 * must not overlap (they share its anchors).
 */
#ifndef TG_ELASTOMER_H
#define TG_ELASTOMER_H
#include <stddef.h>
#include <stdint.h>

#include "tg_proximity.h"
#include "tg_readout.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tg_elast tg_elast; /* opaque: clouds, pads and anchors on the device */

typedef struct {
  uint32_t abi_version;                /* TG_ABI_VERSION */
  int32_t num_envs, num_links, num_taxels, num_objects;
  const int32_t* link_taxel_offset;    /* host [num_links+1]; taxels sorted by link */
  const float* taxel_pos;              /* host [num_taxels][3]  x_j, link frame [m] */
  const float* taxel_normal;           /* host [num_taxels][3]  n_j, unit */
  const float* taxel_radius;           /* host [num_taxels]     R_j of the readout's probes [m] */
  int32_t num_sensor_links;            /* Ls >= 1 */
  const int32_t* sensor_links;         /* host [Ls] link ids, each with 1..64 markers */
  const float* pad_center;             /* host [Ls][3] pad box centre, link frame [m] */
  const float* pad_half;               /* host [Ls][3] pad box half extents [m], > 0 */
  const tg_point_cloud* clouds;        /* host [num_objects], at most 1024 points each */
  float s_d, s_s, lambda_d, lambda_s, alpha, c, eps;   /* App. A.7: 100, 100, 8000, 2000, 1.2, 1,
                                                          eps = the taxel pitch */
  float eta_enter, eta_exit;           /* App. A.7: 1e-5, 1e-4 m */
} tg_elast_config;

/* TG_ERR_INVALID_ARGUMENT for sizes or values outside the ranges above or NULL arrays;
 * TG_ERR_UNSUPPORTED for a sensor link of more than 64 markers, a cloud of more than 1024
 * points, or E * T * 3 beyond 32 bits. */
tg_status tg_elast_create(const tg_elast_config* cfg, tg_elast** out);

/* n_steps consecutive steps in one launch.  in: link_state [n][13][E*L], obj_state [n][13][E] or
 * NULL (objects static at the origin), obj_id [n][E] (-1 or out of range: no object);
 * depth: device [n][E][T], the readout's clean depth of the same steps; disp: device
 * [n][3][E][T], written for the sensor links' markers only (the other entries are left as they
 * are).  Pointers 16-byte aligned. */
tg_status tg_elast_rollout(tg_elast* h, const tg_step_inputs* in, const float* depth, float* disp, int32_t n_steps,
                           void* hip_stream);

/* Clears every anchor and the remembered object of every env (a fill kernel, no memset node). */
tg_status tg_elast_reset(tg_elast* h, void* hip_stream);

tg_status tg_elast_destroy(tg_elast* h); /* NULL is OK */
const char* tg_elast_last_error(const tg_elast* h);

#ifdef __cplusplus
}
#endif
#endif /* TG_ELASTOMER_H */
