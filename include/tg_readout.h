/* tg_readout — batched tactile sensor readout on one MI355X (gfx950).
 *
 * C ABI over device buffers.  The operation is the per-step, per-environment,
 * per-taxel readout of the paper's App. A:
 *   - probe pose q_j = p_L + R_L x_j, a_j = R_L n_j      (App. A.1, probe geometry)
 *   - SDF depth d = [R_j - phi(q_j)]_+ and normal grad phi (App. A.1, sdf backend)
 *   - contact bit with Schmitt hysteresis                 (App. A, ContactProbe)
 *   - raw depth                                            (App. A, ContactDepthProbe)
 *   - six-channel force/torque from depth, normal and
 *     relative velocity                                    (App. A, KinematicTaxel)
 *   - a scalar proximity channel from the SDF              (App. A, ProximityTaxel,
 *     in its flat-surface closed form)
 *   - the noise model: gain, spatial crosstalk, viscoelastic
 *     hysteresis / first-order lag, bias, white noise, random-walk drift,
 *     quantisation, probe-radius noise, dead taxels        (App. A, Sensor Noise Model)
 *   - per-link observations: force/torque sums, contact count,
 *     agg_bool (count > 2) and agg_force                   (App. B, Tactile Observation Types)
 *
 * Conventions shared by every entry point
 *   - Units are SI.  Quaternions are Hamilton (w,x,y,z), used as given (not renormalised).
 *   - "device" pointers are HIP device memory owned by the caller, 16-byte aligned, valid
 *     until the work queued on `hip_stream` has finished.  "host" pointers are read during
 *     the call only and deep-copied where kept.
 *   - Streams are passed as `void*` (a hipStream_t; NULL = the null stream).
 *   - Entry points never throw; they return a tg_status.  On any error nothing is launched
 *     and tg_readout_last_error() describes the failure.
 *   - step/rollout/reset allocate nothing and never synchronise.
 *   - A handle is not thread-safe; use one handle per stream.
 */
#ifndef TG_READOUT_H
#define TG_READOUT_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TG_ABI_VERSION 1u

typedef struct tg_readout tg_readout; /* opaque handle */

typedef enum {
  TG_OK = 0,
  TG_ERR_INVALID_ARGUMENT = 1, /* null/misaligned pointer, bad size or parameter */
  TG_ERR_OUT_OF_MEMORY = 2,    /* device allocation failed in create */
  TG_ERR_HIP = 3,              /* a HIP runtime call failed */
  TG_ERR_UNSUPPORTED = 4,      /* a configuration this library does not implement */
  TG_ERR_UNSTABLE = 5,         /* thermal configuration violates the explicit stability limit */
  TG_ERR_STATE = 6             /* call not valid in the handle's current state */
} tg_status;

/* Output selection bits for tg_readout_config.output_mask. */
enum {
  TG_OUT_BITS = 1u << 0,       /* contact_bits                                   */
  TG_OUT_DEPTH = 1u << 1,      /* depth                                          */
  TG_OUT_PROX = 1u << 2,       /* prox                                           */
  TG_OUT_FT = 1u << 3,         /* ft                                             */
  TG_OUT_NOISY = 1u << 4,      /* ft_noisy + contact_bits_noisy (noise enabled)  */
  TG_OUT_NORMAL = 1u << 5,     /* normal                                         */
  TG_OUT_SURFDIST = 1u << 6,   /* surfdist                                       */
  TG_OUT_LINK_SUMS = 1u << 7,  /* link_sums (+ link_sums_noisy when NOISY)       */
  TG_OUT_TEMP = 1u << 8        /* temperature (thermal fields configured)        */
};

/* One object's signed-distance field sampled on a node-centred cube grid in the object
 * frame: n nodes per axis over [origin, origin + (n-1)*spacing], values x fastest.
 * The readout interpolates it trilinearly and uses the analytic gradient of the same
 * interpolant as the contact normal (App. A.1, sdf backend).  A query outside the box is
 * "far": no contact, no proximity. */
typedef struct {
  int32_t n;           /* >= 2 */
  float origin[3];
  float spacing;       /* > 0 */
  const float* values; /* host, n*n*n floats; deep-copied by create */
} tg_sdf_grid;

/* Noise model (App. A, Sensor Noise Model), applied to the noisy readout only.
 * Order per taxel and channel: gain -> crosstalk -> hysteresis -> + bias + white + drift
 * -> quantisation -> dead overwrite.  Random numbers come from Philox4x32-10 keyed on
 * `seed` with counters (env, taxel, step-derived word, purpose); see tg_readout_reset. */
typedef struct {
  uint64_t seed;
  float drift_sigma;       /* random-walk increment std per step (0 = off)          */
  float white_sigma;       /* additive white noise std (0 = off)                     */
  float bias;              /* constant bias                                          */
  float quant_step;        /* quantisation step q (0 = off): q * rint(x / q)         */
  int32_t hyst_mode;       /* 0 off, 1 first-order lag, 2 single Maxwell element      */
  float tau_load_steps;    /* lag time constant while |x| grows, in steps (> 0)     */
  float tau_unload_steps;  /* lag time constant otherwise, in steps (> 0)           */
  float maxwell_beta;      /* Maxwell strength beta                                  */
  float maxwell_tau_s;     /* Maxwell time constant tau [s] (> 0)                    */
  float dt_s;              /* step length [s]                                        */
  float p_dead;            /* dead-taxel probability, drawn at reset                 */
  float stuck_lo, stuck_hi;/* stuck value of a dead taxel ~ U[lo, hi], drawn at reset */
  float radius_rho;        /* probe-radius noise U[-rho, rho] on the noisy contact bit */
  float gain_lo, gain_hi;  /* per-probe gain ~ U[lo, hi], drawn at reset (1,1 = off) */
  int32_t xtalk_kind;      /* 0 none, 1 banded (chi to each in-link neighbour),
                              2 dense per-link (1-chi) I + chi G_sigma, BF16 on MFMA  */
  float xtalk_chi, xtalk_sigma;
  float eta_off;           /* Schmitt release threshold of the noisy bit (<= eta_on) */
} tg_noise_desc;

/* Voxel temperature fields (App. D, thermal sensing, with the explicit solver of the
 * configuration in place of the paper's spectral one): one 16^3 block per env on each listed
 * link, in that link's frame, voxel edge dx, outer corner of voxel (0,0,0) at `origin`, taxels
 * over the top layer (z index 15).  Per step and voxel, explicit Euler of
 *   rho c_p dT/dt = k lap T + generation + contact conduction - linearised radiation
 * with insulated (mirrored) faces; P_gen spread uniformly over the block; radiation
 * h_r = 4 eps sigma T_amb^3 on every face of the block; contact conduction into the top-layer
 * voxel under each taxel at rate dt pi d_w k_eff d_j / (rho c_p dx^3) per kelvin of
 * (T_obj - T), k_eff = 2 k_sensor k_object / (k_sensor + k_object), d_j the taxel's clean
 * depth.  create returns TG_ERR_UNSTABLE unless 6 r + 3 rho_f + kappa d_max m <= 1 (r =
 * alpha dt / dx^2, rho_f = dt h_r / (rho c_p dx), kappa the contact rate per metre of depth,
 * d_max the largest clean depth the grids allow, m the most taxels over one voxel), which
 * keeps every update a non-negative combination of old temperatures. */
typedef struct {
  int32_t num_fields;            /* thermal links per env (>= 1)                          */
  const int32_t* field_links;    /* host [num_fields], distinct links                     */
  int32_t n;                     /* voxels per axis: 16                                   */
  float dx;                      /* voxel edge [m]                                        */
  float origin[3];               /* link-frame outer corner of voxel (0,0,0) [m]          */
  float dt;                      /* step [s]                                              */
  float k_sensor, rho_cp, emissivity, k_object, d_w;
  float T0, T_amb;               /* initial (at reset) and ambient temperature [degC]     */
  float P_gen;                   /* internal generation per block [W]                     */
  const float* T_obj;            /* host [num_envs] object temperature [degC]; copied     */
  /* solver 1: the paper's own step (App. D.1) instead of the explicit one above.  Per step, in
   * its order: semi-implicit spectral diffusion with zero-flux walls (every mode of the block's
   * mirror extension divided by 1 + alpha dt k^2), the generation, contact conduction as above,
   * then grey-body radiation eps sigma (T_K^4 - T_amb,K^4) and convection h_conv (T - T_amb) per
   * exposed face (divided by rho c_p dx), and the reported temperature passes the sensor
   * element lag T_meas += dt / lag_tau (T - T_meas) (lag_tau <= 0: no lag; the lag state is part
   * of the handle's state, reset to T0).  The diffusion is unconditionally stable; create returns
   * TG_ERR_UNSTABLE unless kappa d_max m <= 1 and 3 (4 eps sigma (T_amb,K + 100)^3 + h_conv) dt /
   * (rho c_p dx) <= 1, and TG_ERR_UNSUPPORTED for a lag on a link of more than 256 taxels. */
  int32_t solver;                /* 0 explicit (default), 1 the paper's spectral step    */
  float h_conv;                  /* convection coefficient [W/m^2K] (solver 1)            */
  float lag_tau;                 /* sensor element time constant [s] (solver 1)           */
} tg_thermal_desc;

typedef struct {
  uint32_t abi_version;            /* TG_ABI_VERSION */
  int32_t num_envs, num_links, num_taxels, num_objects;
  const int32_t* link_taxel_offset;/* host [num_links+1]; taxels sorted by link; a link
                                      may be empty (offset[l+1] == offset[l]): its link
                                      sums are zero                                       */
  const float* taxel_pos;          /* host [num_taxels*3] link-frame x_j [m]              */
  const float* taxel_normal;       /* host [num_taxels*3] link-frame unit n_j             */
  const float* taxel_radius;       /* host [num_taxels] R_j [m]; 0 = inactive filler      */
  const tg_sdf_grid* grids;        /* host [num_objects]                                  */
  float k_n, c_n, alpha, k_t, k_w, mu; /* KinematicTaxel law, Coulomb cap mu            */
  float prox_range;                /* proximity range R_p [m]                             */
  float eta_on;                    /* contact threshold [m]                               */
  int32_t ft_spring_only;          /* 1: f = k_n d^alpha m_bar, tau = x_j x f             */
  int32_t noise_enabled;
  tg_noise_desc noise;
  uint32_t output_mask;            /* TG_OUT_* bits                                       */
  /* SDF backend.  0: the grids (App. A.1, sdf backend).  1: per-object neural surrogates
   * (include/tg_nsdf.h network and parameter layout) with the grid as fallback wherever the
   * probe centre is outside the object's grid box or |phi_nn| < nsdf_band; the normal comes
   * from the network's input gradient outside the band.  Mode 1 computes the clean outputs
   * only (noise_enabled must be 0). */
  int32_t sdf_mode;
  float nsdf_band;                 /* [m], >= 0 (mode 1)                                   */
  const float* nsdf_params;        /* device [num_objects][15681] FP32; read during create
                                      only (packed into library-owned BF16 images)          */
  const tg_thermal_desc* thermal;  /* NULL = no thermal fields (requires sdf_mode 0)       */
} tg_readout_config;

/* Per-step inputs, device, SoA.  For tg_readout_rollout each array holds n_steps
 * consecutive copies of the one-step layout. */
typedef struct {
  const float* link_state;  /* [13][num_envs*num_links]: px py pz qw qx qy qz vx vy vz wx wy wz,
                               column e*num_links + l; world frame, velocities at the link origin */
  const float* obj_state;   /* [13][num_envs] same layout for the object, or NULL: object static
                               at the env origin with identity orientation                      */
  const int32_t* obj_id;    /* [num_envs]; -1 (or out of range) = no object in contact          */
  int64_t step;             /* global index of the first step: RNG counter and Schmitt clock,
                               0 <= step < 2^32                                                 */
} tg_step_inputs;

/* Per-step outputs, device, caller-owned; a pointer must be non-NULL iff its output is
 * selected in output_mask.  Rollouts write n_steps consecutive copies. */
typedef struct {
  uint64_t* contact_bits;        /* [E][ceil(T/64)]: bit j%64 of word j/64 = (d > eta_on)  */
  uint64_t* contact_bits_noisy;  /* [E][ceil(T/64)]                                        */
  float* depth;                  /* [E][T] d [m]                                           */
  float* prox;                   /* [E][T] proximity in [0,1]                              */
  float* surfdist;               /* [E][T] SDF at the probe centre [m] (FLT_MAX if none)  */
  float* ft;                     /* [6][E][T] fx fy fz tx ty tz, link frame                */
  float* ft_noisy;               /* [6][E][T]                                              */
  float* normal;                 /* [3][E][T] link-frame contact normal (0 if no contact)  */
  float* link_sums;              /* [11][L][E] sum f(3), sum tau(3), count, agg_bool,
                                    agg_force = 1e4 (sum d n_z, sum d n_y, sum d n_x);
                                    env-innermost, so a workgroup's envs of one link are
                                    contiguous (App. B.2 per-link observations)            */
  float* link_sums_noisy;        /* [11][L][E] same on the noisy channel                   */
  float* temperature;            /* [E][T] after the step: temperature of the top-layer voxel
                                    under each taxel of a thermal link, 0 elsewhere         */
} tg_step_outputs;

/* Create a handle: validates the configuration, deep-copies every host array to device
 * memory (grids, taxel constants, crosstalk blocks), allocates the noise state and runs
 * tg_readout_reset(all envs, step 0).  *out is NULL on error. */
tg_status tg_readout_create(const tg_readout_config* cfg, tg_readout** out);

/* One step for every env on `hip_stream`.  Equivalent to tg_readout_rollout(h, in, out, 1, s). */
tg_status tg_readout_step(tg_readout* h, const tg_step_inputs* in, const tg_step_outputs* out,
                          void* hip_stream);

/* n_steps consecutive steps (in->step, in->step+1, ...) in one persistent launch: the noise
 * state stays on chip between steps.  n_steps = 0 is a no-op returning TG_OK. */
tg_status tg_readout_rollout(tg_readout* h, const tg_step_inputs* in, const tg_step_outputs* out,
                             int32_t n_steps, void* hip_stream);

/* Episode reset (App. A noise model: gain, dead taxels and stuck values are drawn at reset;
 * drift, hysteresis and Schmitt state return to zero).  env_mask_dev: device uint8[E],
 * nonzero = reset that env; NULL = all envs.  The draws use counter (env, taxel, step, 7). */
tg_status tg_readout_reset(tg_readout* h, const uint8_t* env_mask_dev, int64_t step, void* hip_stream);

/* Size in bytes of the dynamic state: noise state (drift, hysteresis, Schmitt, dead, stuck,
 * gain) followed, with thermal fields, by the fields as float [E][num_fields][16][16][16]
 * (index ((z * 16) + y) * 16 + x, degC).  Reset sets the fields of the reset envs to T0. */
tg_status tg_readout_state_size(const tg_readout* h, size_t* bytes);
/* Copy the noise state to / from a device buffer of tg_readout_state_size bytes (checkpoint). */
tg_status tg_readout_get_state(tg_readout* h, void* dst_dev, size_t bytes, void* hip_stream);
tg_status tg_readout_set_state(tg_readout* h, const void* src_dev, size_t bytes, void* hip_stream);

/* Errors found on the device, where the host cannot check inputs without a synchronisation
 * (the boundary's convention for device-resident values).  Waits for all device work, returns
 * the accumulated flags in *device_error_flags and clears them:
 *   TG_DEVERR_BAD_OBJECT_ID  an object id outside [-1, num_objects) was read; that env was read
 *                            out as having no object (every output zero), as for id -1.
 * TG_ERR_INVALID_ARGUMENT for a NULL handle or flags pointer. */
#define TG_DEVERR_BAD_OBJECT_ID 1u
tg_status tg_readout_poll_errors(tg_readout* h, uint32_t* device_error_flags);

/* Kernel launch shape the handle uses (for profiling tools): envs per block and threads. */
tg_status tg_readout_launch_shape(const tg_readout* h, int32_t* envs_per_block, int32_t* threads);

/* Graph mode (default on): rollout records its kernel launches once into a HIP graph on a
 * private stream and replays the graph on `hip_stream`, updating only the launch arguments on
 * later calls.  When `hip_stream` is itself being captured the plain launches are issued
 * instead, so a caller can capture rollout into its own graph. */
tg_status tg_readout_set_graph(tg_readout* h, int32_t enable);

/* Autotuner for the readout kernel's work plan: readouts per workgroup 128, 192, 256, 320, 384,
 * 448, 512 (one link per workgroup, so this sets the envs per workgroup and with them the waves
 * per workgroup).  Runs each candidate on the caller's inputs and outputs for n_steps steps,
 * keeps the fastest plan for this handle and reports it.  Unlike step/rollout it allocates a
 * state buffer, synchronises and overwrites `out`; the dynamic state is restored afterwards.
 * The result is cached for the process under a hash of the configuration (sizes, link layout,
 * grid sizes, noise kernel variant, output mask, backend, thermal fields), n_steps and whether
 * objects move: a later call with the same key, on any handle, applies the cached plan without
 * timing and touches neither `out` nor the state.  The neural backend has no plan to tune
 * (best_target = 0). */
tg_status tg_readout_autotune(tg_readout* h, const tg_step_inputs* in, const tg_step_outputs* out, int32_t n_steps,
                              void* hip_stream, int32_t* best_target, float* best_ms);

/* Fix the readout kernel's work plan without timing: about `readouts_per_workgroup` readouts
 * (64..1024) per workgroup, as the autotuner would set it.  Synchronises the device.  Returns
 * TG_ERR_INVALID_ARGUMENT for a size outside 64..1024 or a plan whose LDS exceeds the 160 KiB of
 * a gfx950 CU, TG_ERR_UNSUPPORTED for one that needs more than 512 threads per workgroup; the
 * previous plan is then kept.  The neural backend has no plan (no-op). */
tg_status tg_readout_set_work_plan(tg_readout* h, int32_t readouts_per_workgroup);

/* Release the handle and its device memory (synchronises the device). NULL is accepted. */
tg_status tg_readout_destroy(tg_readout* h);

/* Message of the last error on this handle ("" if none); NULL handle: last create error. */
const char* tg_readout_last_error(const tg_readout* h);
const char* tg_status_string(tg_status s);

#ifdef __cplusplus
}
#endif
#endif
