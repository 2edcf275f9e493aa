/* CPU oracle for the tactile readout.  TEST INFRASTRUCTURE ONLY: the product
 * path never includes, links or calls anything in this directory.
 *
 * A plain, slow, step-by-step implementation of the readout defined in the
 * paper's App. A (probe geometry, SDF depth backend, ContactProbe,
 * ContactDepthProbe, KinematicTaxel, the proximity channel) and App. A noise
 * model, plus the observation post-processing of App. B (agg_bool,
 * agg_force).  It is built twice from one source (oracle_impl.h): with
 * REAL = float it follows the written FP32 operation sequence and is the
 * parity oracle; with REAL = double it is the FP64 reference used for error
 * reports and closed-form pins.
 */
#ifndef TG_ORACLE_H
#define TG_ORACLE_H
#include <stdint.h>

typedef struct {
  int32_t n;              /* nodes per axis; 0 selects the analytic sphere below (pins only) */
  float origin[3];        /* object-frame position of node (0,0,0) */
  float spacing;          /* node spacing h */
  const float* values;    /* [n][n][n], x fastest */
  double sphere_c[3];     /* analytic sphere centre and radius when n == 0 */
  double sphere_r;
} or_grid;

typedef struct {
  int32_t num_envs;            /* envs in this batch */
  const int32_t* env_index;    /* [num_envs] global env ids (RNG counters); NULL = 0..E-1 */
  int32_t num_links, num_taxels, num_objects;
  const int32_t* link_offset;  /* [L+1] */
  const float* taxel_pos;      /* [T][3] */
  const float* taxel_normal;   /* [T][3] */
  const float* taxel_radius;   /* [T] */
  const or_grid* grids;        /* [num_objects] */
  float k_n, c_n, alpha, k_t, k_w, mu, prox_range, eta_on;
  int32_t spring_only;
  int32_t noise_on;
  uint64_t seed;
  float drift_sigma, white_sigma, bias, quant_step;
  int32_t hyst_mode;           /* 0 off, 1 asymmetric lag, 2 Maxwell element */
  float tau_load, tau_unload, maxwell_beta, maxwell_tau, dt;
  float p_dead, stuck_lo, stuck_hi, radius_rho, gain_lo, gain_hi;
  int32_t xtalk_kind;          /* 0 none, 1 banded, 2 dense */
  float xtalk_chi, xtalk_sigma;
  float eta_off;
  /* SDF backend: 0 = grids; 1 = per-object neural surrogate (or_nsdf_forward with BF16
   * emulation) wherever the probe centre is inside the grid box and |phi_nn| >= nsdf_band,
   * the grid elsewhere. */
  int32_t sdf_mode;
  float nsdf_band;
  const double* nsdf_params;   /* [num_objects][15681] */
} or_problem;

typedef struct {
  const float* link_state;     /* [S][13][E*L] */
  const int32_t* obj_id;       /* [S][E] */
  const float* obj_state;      /* [S][13][E] or NULL */
  int64_t step0;
  int32_t num_steps;
} or_inputs;

typedef struct {               /* every array [S][...]; NULL = not produced */
  uint8_t* bit;                /* [S][E][T] */
  uint8_t* bit_noisy;          /* [S][E][T] */
  double* depth;               /* [S][E][T] */
  double* prox;                /* [S][E][T] */
  double* surfdist;            /* [S][E][T] */
  double* ft;                  /* [S][6][E][T] */
  double* ft_noisy;            /* [S][6][E][T] */
  double* normal;              /* [S][3][E][T] */
  double* link_sums;           /* [S][11][E][L] */
  double* link_sums_noisy;     /* [S][11][E][L] */
  double* xtalk_scale;         /* [S][6][E][T]: sum_k |C_jk||z_k| of the crosstalk sum */
  double* xhat;                /* [S][3][E][T]: the network's input x_hat where the neural backend
                                  evaluated it, NaN elsewhere (a record, for diagnostics) */
} or_outputs;

typedef struct {
  double* drift;               /* [6][E][T] */
  double* hyst;                /* [6][E][T] lag output y, or Maxwell xi */
  double* hyst_prev;           /* [6][E][T] Maxwell previous input */
  uint8_t* schmitt;            /* [E][T] */
  uint8_t* dead;               /* [E][T] */
  double* stuck;               /* [E][T] */
  double* gain;                /* [E][T] */
} or_state;

/* Thermal fields (App. D, thermal sensing; explicit voxel solver): one n^3 field per env on each
 * listed link, in that link's frame.  Temperatures in degC. */
typedef struct {
  int32_t num_fields;          /* fields per env */
  const int32_t* field_link;   /* [num_fields] link of each field */
  int32_t n;                   /* voxels per axis */
  float dx;                    /* voxel edge [m] */
  float origin[3];             /* link-frame position of the outer corner of voxel (0,0,0) */
  float dt;                    /* [s] */
  float k_sensor, rho_cp, emissivity, k_object, d_w;
  float T0, T_amb;             /* initial and ambient temperature */
  float P_gen;                 /* uniform internal generation per field [W] */
  const float* T_obj;          /* [E] object temperature per env */
} or_thermal;

typedef struct {               /* derived constants, FP64 */
  double alpha, r, h_r, rho_f, g, k_eff, kappa;
} or_thermal_consts;

#ifdef __cplusplus
extern "C" {
#endif
void or_thermal_constants(const or_thermal* th, or_thermal_consts* K);
int or_thermal_voxel(const or_thermal* th, const float* x);
int or_thermal_stable(const or_thermal* th, double delta_max, int32_t taxels_per_voxel_max);
int or_thermal_run_f32(const or_thermal* th, int32_t E, int32_t T, const int32_t* link_offset, const float* taxel_pos,
                       const double* depth, int32_t S, float* fields, double* taxel_temp, double* ledger);
int or_thermal_run_f64(const or_thermal* th, int32_t E, int32_t T, const int32_t* link_offset, const float* taxel_pos,
                       const double* depth, int32_t S, double* fields, double* taxel_temp, double* ledger);
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int or_reset_f32(const or_problem* P, or_state* st, const uint8_t* env_mask, int64_t reset_step);
int or_reset_f64(const or_problem* P, or_state* st, const uint8_t* env_mask, int64_t reset_step);
int or_run_f32(const or_problem* P, const or_inputs* in, or_outputs* out, or_state* st, int threads);
int or_run_f64(const or_problem* P, const or_inputs* in, or_outputs* out, or_state* st, int threads);
int or_dense_xtalk_f64(const or_problem* P, double* out);  /* concat of n_l*n_l, row-major */
float or_bf16_round(float x);
void or_nsdf_forward(const double* P, int64_t n, const double* x, double* out, double* gx, int bf16);
#ifdef __cplusplus
}
#endif
#endif
