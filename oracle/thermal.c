/* Thermal field oracle (explicit 7-point voxel solver with sources).  TEST INFRASTRUCTURE ONLY.
 * Definitions in thermal_impl.h; built for REAL = float (parity) and REAL = double (pins). */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* Derived constants (FP64): alpha = k / (rho c_p); r = alpha dt / dx^2;
 * h_r = 4 eps sigma (T_amb + 273.15)^3 (radiation linearised about the ambient);
 * rho_f = dt h_r / (rho c_p dx) per exposed face; g = dt P_gen / (n^3 rho c_p dx^3);
 * k_eff = 2 k_s k_o / (k_s + k_o) (series conductance of sensor and object);
 * kappa = dt pi d_w k_eff / (rho c_p dx^3) per metre of depth. */
void or_thermal_constants(const or_thermal* th, or_thermal_consts* K) {
  const double dx = th->dx, rc = th->rho_cp, dt = th->dt;
  const double sigma_sb = 5.670374419e-8;
  const double Ta = (double)th->T_amb + 273.15;
  K->alpha = (double)th->k_sensor / rc;
  K->r = K->alpha * dt / (dx * dx);
  K->h_r = 4.0 * (double)th->emissivity * sigma_sb * Ta * Ta * Ta;
  K->rho_f = dt * K->h_r / (rc * dx);
  K->g = dt * (double)th->P_gen / ((double)th->n * th->n * th->n * rc * dx * dx * dx);
  K->k_eff = 2.0 * (double)th->k_sensor * (double)th->k_object / ((double)th->k_sensor + (double)th->k_object);
  K->kappa = dt * M_PI * (double)th->d_w * K->k_eff / (rc * dx * dx * dx);
}

/* Top-layer voxel (index y * n + x) under a taxel at link-frame position x (clamped into the block). */
int or_thermal_voxel(const or_thermal* th, const float* x) {
  int idx[2];
  for (int d = 0; d < 2; ++d) {
    int i = (int)floor(((double)x[d] - (double)th->origin[d]) / (double)th->dx);
    i = i < 0 ? 0 : (i > th->n - 1 ? th->n - 1 : i);
    idx[d] = i;
  }
  return idx[1] * th->n + idx[0];
}

/* Explicit-step positivity: every voxel's new value is a non-negative combination of old values
 * and source temperatures when 6 r + 3 rho_f + kappa * delta_max * m <= 1 (m = most taxels over one
 * voxel, delta_max = largest possible clean depth).  Returns 1 when the bound holds. */
int or_thermal_stable(const or_thermal* th, double delta_max, int32_t taxels_per_voxel_max) {
  or_thermal_consts K;
  or_thermal_constants(th, &K);
  return 6.0 * K.r + 3.0 * K.rho_f + K.kappa * delta_max * (double)taxels_per_voxel_max <= 1.0;
}

#define REAL float
#define SFX(name) name##_f32
#include "thermal_impl.h"
#undef REAL
#undef SFX

#define REAL double
#define SFX(name) name##_f64
#include "thermal_impl.h"
#undef REAL
#undef SFX
