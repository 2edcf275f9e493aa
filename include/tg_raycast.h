/* tg_raycast — the raycast contact-depth backend (App. A.1) on one MI355X (gfx950).
 *
 * The alternative to the SDF backend: the contact depth of each probe comes from the object's
 * triangle mesh through a bounding-volume hierarchy.  Probe j of link L has centre
 * q_j = p_L + R_L x_j, axis a_j = R_L n_j (pointing toward the object) and radius R_j; the mesh is
 * closed with outward faces, in the object's frame.  Per triangle:
 *   - sphere test: R_j - (distance from q_j to the triangle's closest point);
 *   - ray test: a ray from q_j along -a_j; when its first crossing with the mesh leaves the mesh
 *     (the crossed face's outward normal has a positive component along the ray), q_j is inside
 *     the object and the penetration is R_j + t (t the distance to that face), R_j minus the
 *     hit's signed distance along a_j.
 * The deepest penetration wins; the depth is its positive part and the contact normal the
 * outward normal of the winning face, in the link frame.  A probe with R_j = 0 reads zero.  For
 * probe centres outside the object this is R_j - phi; inside it is R_j + (the distance along the
 * axis to the surface), R_j - phi to leading order for faces facing the probe.
 *
 * The library builds one BVH per object at create (median splits on the longest axis of the
 * triangle centroids, at most 4 triangles per leaf).  One thread per (step, env, probe) traverses
 * it twice: a sphere query whose radius shrinks as the best penetration grows, then a closest-hit
 * ray query, both nearer child first.  Geometry is FP32.
 *
 * Conventions are those of tg_readout.h: create deep-copies the host arrays; device buffers are
 * caller-owned and must stay valid until the queued work finishes; calls return a tg_status and
 * launch nothing on error; rollout allocates nothing and never synchronises.
 */
#ifndef TG_RAYCAST_H
#define TG_RAYCAST_H
#include <stddef.h>
#include <stdint.h>

#include "tg_readout.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tg_ray tg_ray; /* opaque: per-object BVHs and triangles on the device */

typedef struct {
  int32_t num_verts;      /* >= 3 */
  const float* verts;     /* host [num_verts][3], object frame [m] */
  int32_t num_tris;       /* >= 1 */
  const int32_t* tris;    /* host [num_tris][3] vertex indices, counter-clockwise seen from outside */
} tg_mesh;

typedef struct {
  uint32_t abi_version;                /* TG_ABI_VERSION */
  int32_t num_envs, num_links, num_taxels, num_objects;
  const int32_t* link_taxel_offset;    /* host [num_links+1]; taxels sorted by link */
  const float* taxel_pos;              /* host [num_taxels][3]  x_j, link frame [m] */
  const float* taxel_normal;           /* host [num_taxels][3]  n_j, unit */
  const float* taxel_radius;           /* host [num_taxels]     R_j [m], >= 0 */
  const tg_mesh* meshes;               /* host [num_objects], closed, outward faces */
} tg_ray_config;

/* TG_ERR_INVALID_ARGUMENT for non-positive sizes, NULL arrays, a vertex index out of range, a
 * degenerate triangle or a non-finite vertex; TG_ERR_UNSUPPORTED when E * T * 3 does not fit 32
 * bits or a mesh has more than 2^20 triangles. */
tg_status tg_ray_create(const tg_ray_config* cfg, tg_ray** out);

/* n_steps consecutive steps in one launch.  in: link_state [n][13][E*L], obj_state [n][13][E] or
 * NULL (objects static at the origin), obj_id [n][E] (-1 or out of range: no object, depth 0).
 * depth: device [n][E][T]; normal: device [n][3][E][T] (link frame, 0 without contact) or NULL;
 * tri: device [n][E][T] int32, the winning triangle's index in its mesh (-1 without contact), or
 * NULL.  Pointers 16-byte aligned. */
tg_status tg_ray_rollout(tg_ray* h, const tg_step_inputs* in, float* depth, float* normal, int32_t* tri,
                         int32_t n_steps, void* hip_stream);

tg_status tg_ray_destroy(tg_ray* h); /* NULL is OK */
const char* tg_ray_last_error(const tg_ray* h);

#ifdef __cplusplus
}
#endif
#endif /* TG_RAYCAST_H */
