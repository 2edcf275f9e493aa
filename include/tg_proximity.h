/* tg_proximity — the ProximityTaxel readout (App. A.6) on one MI355X (gfx950).
 *
 * A proximity taxel responds to the tracked object's surface mass inside its sensing sphere, the
 * way capacitive and magnetic skins do.  Each object carries a surface point cloud p_hat_i in its
 * own frame (sampled once, at scene reset, by the caller); in the world p_i = R_O p_hat_i + p_O.
 * For taxel j on link L, with probe centre q_j = p_L + R_L x_j, axis a_j = R_L n_j and sensing
 * radius R_j (App. A.6 definitions):
 *   P_ij = R_j - |p_i - q_j|  over the points with |p_i - q_j| < R_j            (penetration)
 *   v_tax = v_L + w_L x (q_j - p_L),  v_p_i = v_O + w_O x (p_i - p_O)            (point velocities)
 *   v_t,ij = (v_p_i - v_tax) - a_j ((v_p_i - v_tax) . a_j)                       (normal part removed)
 *   rho_b = density / max(N_active_b, 1)   (N_active_b: points of env b's object; 0 without one)
 *   f = k rho_b sum P_ij a_j + k_s rho_b sum P_ij v_t,ij,   tau = k rho_b sum P_ij (p_i - q_j) x a_j
 * and the six channels are R_L^T f and R_L^T tau.  Radius noise perturbs R_j before the query:
 * R_j + radius_rho (2u - 1), u = (2 (x >> 9) + 1) 2^-24 with x the first word of Philox4x32-10,
 * key = seed, counter (env, taxel, step, 9); a per-probe gain (optional) scales the six channels.
 *
 * The library keeps each cloud in a uniform cell grid in the object frame (cell edge = half the
 * largest sensing radius plus radius_rho), points sorted by cell, so a query visits, in each row of
 * cells its sphere reaches, the cells under the sphere's chord as one contiguous run of points;
 * the sums above are formed from two moments
 * accumulated over the visited points, sum P_ij and sum P_ij (p_i - q_j), which give every term of
 * f and tau (the velocity of a point is affine in its position).
 *
 * Conventions are those of tg_readout.h: create deep-copies the host arrays; device buffers are
 * caller-owned and must stay valid until the queued work finishes; calls return a tg_status,
 * launch nothing on error, allocate nothing and never synchronise after create.
 */
#ifndef TG_PROXIMITY_H
#define TG_PROXIMITY_H
#include <stddef.h>
#include <stdint.h>

#include "tg_readout.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tg_prox tg_prox; /* opaque: cell grids and sorted clouds on the device */

typedef struct {
  int32_t num_points;   /* >= 0 */
  const float* points;  /* host [num_points][3], object frame [m] */
} tg_point_cloud;

typedef struct {
  uint32_t abi_version;                /* TG_ABI_VERSION */
  int32_t num_envs, num_links, num_taxels, num_objects;
  const int32_t* link_taxel_offset;    /* host [num_links+1]; taxels sorted by link */
  const float* taxel_pos;              /* host [num_taxels][3]  x_j, link frame [m] */
  const float* taxel_normal;           /* host [num_taxels][3]  n_j, unit */
  const float* sensing_radius;         /* host [num_taxels]     R_j [m], >= 0 */
  const tg_point_cloud* clouds;        /* host [num_objects] */
  float k, k_s, density;               /* App. A.6 settings: 300, 10, 100 */
  uint64_t seed;                       /* Philox key of the radius noise */
  float radius_rho;                    /* radius noise half-width [m]; 0 = off */
} tg_prox_config;

/* TG_ERR_INVALID_ARGUMENT for non-positive sizes, NULL arrays, a negative radius or a cloud
 * with NULL points; TG_ERR_UNSUPPORTED when num_envs * num_taxels * 6 does not fit 32 bits. */
tg_status tg_prox_create(const tg_prox_config* cfg, tg_prox** out);

/* n_steps consecutive steps in one launch.  in: link_state [n_steps][13][E*L], obj_state
 * [n_steps][13][E] or NULL (objects static at the origin), obj_id [n_steps][E] (-1 or out of range:
 * no object, all channels 0), in->step the first step's index (radius noise counter).
 * ft: device [n_steps][6][E][T] (fx fy fz tx ty tz, link frame); mass: device [n_steps][E][T]
 * (sum_i P_ij) or NULL; gain: device [E][T] or NULL (1).  Pointers 16-byte aligned. */
tg_status tg_prox_rollout(tg_prox* h, const tg_step_inputs* in, float* ft, float* mass, const float* gain,
                          int32_t n_steps, void* hip_stream);

tg_status tg_prox_destroy(tg_prox* h); /* NULL is OK */
const char* tg_prox_last_error(const tg_prox* h);

#ifdef __cplusplus
}
#endif
#endif /* TG_PROXIMITY_H */
