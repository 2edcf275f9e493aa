/* Thermal field oracle body, instantiated for REAL = float and REAL = double (see thermal.c).
 * TEST INFRASTRUCTURE ONLY.
 *
 * Per field (one per env and thermal link), per step, explicit Euler of
 *   rho c_p dT/dt = k lap T + q_gen + q_contact - q_rad
 * on an n^3 voxel grid in the link frame (App. D, thermal sensing; the paper's spectral solver
 * is replaced by the explicit 7-point stencil of the configuration), with:
 *   - diffusion: r * (sum of the 6 neighbours - 6 T), r = alpha dt / dx^2, insulated (Neumann)
 *     faces by mirroring (a missing neighbour takes the voxel's own value);
 *   - generation: g = dt P_gen / (n^3 rho c_p dx^3) in every voxel;
 *   - radiation, linearised about the ambient: rho_f * faces * (T_amb - T) on every voxel with
 *     `faces` faces on the block surface, rho_f = dt h_r / (rho c_p dx), h_r = 4 eps sigma T_amb^3;
 *   - contact conduction into the top-layer voxel under each taxel of the link:
 *     c_v * (T_obj - T), c_v = kappa * sum of the clean depths of the taxels over voxel v,
 *     kappa = dt pi d_w k_eff / (rho c_p dx^3), k_eff = 2 k_s k_o / (k_s + k_o).
 * FP32 sequence (both the oracle's float build and the library):
 *   s   = ((T[x-1] + T[x+1]) + (T[y-1] + T[y+1])) + (T[z-1] + T[z+1])
 *   src = (g + rho_f * faces * (T_amb - T)) + c_v * (T_obj - T)
 *   T'  = T + (r * (s - 6 T) + src)
 * with faces * rho_f and the constants precomputed, c_v summed in taxel order.
 */

static void SFX(th_step)(const or_thermal* th, const or_thermal_consts* K, const REAL* T, REAL* Tn, const REAL* cv,
                         REAL Tobj, double* e_store, double* e_src) {
  const int n = th->n;
  const REAL r = (REAL)K->r, g = (REAL)K->g, rf = (REAL)K->rho_f, Tamb = (REAL)th->T_amb;
  double es = 0, ei = 0;
  const double vol_cap = (double)th->rho_cp * (double)th->dx * (double)th->dx * (double)th->dx;
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const int64_t i = ((int64_t)z * n + y) * n + x;
        const REAL t = T[i];
        const REAL xm = x > 0 ? T[i - 1] : t, xp = x < n - 1 ? T[i + 1] : t;
        const REAL ym = y > 0 ? T[i - n] : t, yp = y < n - 1 ? T[i + n] : t;
        const REAL zm = z > 0 ? T[i - n * n] : t, zp = z < n - 1 ? T[i + n * n] : t;
        const REAL s = ((xm + xp) + (ym + yp)) + (zm + zp);
        const int faces = (x == 0) + (x == n - 1) + (y == 0) + (y == n - 1) + (z == 0) + (z == n - 1);
        const REAL rfx = rf * (REAL)faces;
        REAL src = g + rfx * (Tamb - t);
        const REAL c = z == n - 1 ? cv[y * n + x] : (REAL)0;
        src = src + c * (Tobj - t);
        const REAL tn = t + (r * (s - (REAL)6 * t) + src);
        Tn[i] = tn;
        es += vol_cap * ((double)tn - (double)t);
        ei += vol_cap * (double)src;
      }
  *e_store += es;
  *e_src += ei;
}

/* fields: [E][F][n^3] (in: state, out: state after S steps); depth: [S][E][T] clean depths;
 * taxel_temp: [S][E][T] (temperature of the voxel under each thermal taxel after the step, 0
 * elsewhere) or NULL; ledger: [S][E][F][2] (stored energy change, source energy) or NULL. */
int SFX(or_thermal_run)(const or_thermal* th, int32_t E, int32_t T, const int32_t* link_offset, const float* taxel_pos,
                        const double* depth, int32_t S, REAL* fields, double* taxel_temp, double* ledger) {
  or_thermal_consts K;
  or_thermal_constants(th, &K);
  const int n = th->n, F = th->num_fields;
  const int64_t NV = (int64_t)n * n * n;
  int* vox = (int*)malloc(sizeof(int) * (size_t)T);
  for (int j = 0; j < T; ++j) vox[j] = -1;
  for (int f = 0; f < F; ++f) {
    const int l = th->field_link[f];
    for (int j = link_offset[l]; j < link_offset[l + 1]; ++j) vox[j] = or_thermal_voxel(th, taxel_pos + 3 * j);
  }
  REAL* tmp = (REAL*)malloc(sizeof(REAL) * (size_t)NV);
  REAL* cv = (REAL*)malloc(sizeof(REAL) * (size_t)n * n);
  const REAL kap = (REAL)K.kappa;
  for (int s = 0; s < S; ++s) {
    if (taxel_temp) memset(taxel_temp + (int64_t)s * E * T, 0, sizeof(double) * (size_t)E * T);
    for (int e = 0; e < E; ++e) {
      const REAL Tobj = (REAL)th->T_obj[e];
      for (int f = 0; f < F; ++f) {
        const int l = th->field_link[f];
        REAL* fld = fields + ((int64_t)e * F + f) * NV;
        for (int v = 0; v < n * n; ++v) cv[v] = 0;
        for (int j = link_offset[l]; j < link_offset[l + 1]; ++j) {
          const REAL d = (REAL)depth[((int64_t)s * E + e) * T + j];
          cv[vox[j]] = cv[vox[j]] + kap * d;
        }
        double es = 0, ei = 0;
        SFX(th_step)(th, &K, fld, tmp, cv, Tobj, &es, &ei);
        memcpy(fld, tmp, sizeof(REAL) * (size_t)NV);
        if (ledger) {
          ledger[(((int64_t)s * E + e) * F + f) * 2] = es;
          ledger[(((int64_t)s * E + e) * F + f) * 2 + 1] = ei;
        }
        if (taxel_temp)
          for (int j = link_offset[l]; j < link_offset[l + 1]; ++j)
            taxel_temp[((int64_t)s * E + e) * T + j] = (double)fld[(int64_t)(n - 1) * n * n + vox[j]];
      }
    }
  }
  free(vox);
  free(tmp);
  free(cv);
  return 0;
}
